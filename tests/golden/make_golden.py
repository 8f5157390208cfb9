"""Write the FP64-oracle expected values used by the full-size GPU parity tests.

Calls only ``oracle/`` (bucket elimination with its own min-fill orders, in
double complex) on seeded synthetic instances from ``qaoa_synth``; no value
comes from the HIP library.

    python tests/golden/make_golden.py cfg2 [threads]
    python tests/golden/make_golden.py cfg3 [threads]
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import qaoa_synth as qs  # noqa: E402

CASES = {
    # random 3-regular N=30, depth 4 (the paper's Sec. II-E benchmark shape)
    "cfg2": dict(n=30, d=3, p=4, seed=0, angle_set=0),
    # random 4-regular N=40, depth 3
    "cfg4": dict(n=40, d=4, p=3, seed=0, angle_set=0),
}

# The batched set: 64 cubic graphs, N even in [20, 200], p in {2, 3, 4}.
BATCH = dict(master_seed=2204, count=64, n_lo=20, n_hi=200, depths=(2, 3, 4), d=3)
# Graphs whose whole energy the oracle evaluates: every graph whose light
# cones sum to at most this many 2^width units (all depth-2 and depth-3
# graphs and the lighter depth-4 ones).
BATCH_FULL_COST = 7e8
# Of every heavier graph, the oracle evaluates the light cones of the largest
# width at most BATCH_MAX_WIDTH (all of them; memory: one width-30 bucket
# holds 2^29 complex128 values, 8 GiB) and its cheapest one.
BATCH_MAX_WIDTH = 30


def make(name, threads):
    c = CASES[name]
    inst = qs.instance(c["n"], c["d"], c["p"], c["seed"], c["angle_set"] + 1)
    gamma, beta = inst["angles"][c["angle_set"]]
    t0 = time.time()
    zz, energy = oracle.energy(c["n"], inst["edges"], gamma, beta, threads=threads)
    out = {
        "case": name, **c,
        "edges": [list(e) for e in inst["edges"]],
        "gamma": gamma, "beta": beta,
        "zz_re": [float(z.real) for z in zz],
        "zz_im": [float(z.imag) for z in zz],
        "energy": energy,
        "oracle": "FP64 bucket elimination, greedy min-fill per light cone",
        "oracle_seconds": round(time.time() - t0, 1),
        "threads": threads,
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["energy"], out["oracle_seconds"], "s")


def instance_digest(inst):
    """Digest of a batched instance's edges and first angle set, so that a
    reader can tell that it regenerated the same graph."""
    h = hashlib.sha256()
    h.update(json.dumps([list(e) for e in inst["edges"]]).encode())
    g, b = inst["angles"][0]
    h.update(json.dumps([list(map(float, g)), list(map(float, b))]).encode())
    return h.hexdigest()[:16]


def make_batch(threads):
    b = BATCH
    insts = qs.batch_instances(b["master_seed"], b["count"], b["n_lo"], b["n_hi"],
                               b["depths"], d=b["d"])
    graphs = []
    t_all = time.time()
    for gi, it in enumerate(insts):
        n, edges, p = it["n"], it["edges"], it["p"]
        g, bt = it["angles"][0]
        widths = [[int(x) for x in oracle.edge_widths(n, edges, k, p)] for k in range(len(edges))]
        cost = [sum(2.0 ** x for x in w if x) for w in widths]
        wmax = [max(w) for w in widths]
        rec = {"index": gi, "n": n, "p": p, "m": len(edges), "digest": instance_digest(it)}
        t0 = time.time()
        if sum(cost) <= BATCH_FULL_COST:
            zz, energy = oracle.energy(n, edges, g, bt, threads=threads)
            rec.update(edge_ids=list(range(len(edges))), energy=energy)
        else:
            ok = [k for k in range(len(edges)) if wmax[k] <= BATCH_MAX_WIDTH]
            top = max(wmax[k] for k in ok)
            cheapest = min(range(len(edges)), key=lambda k: cost[k])
            sel = sorted({k for k in ok if wmax[k] == top} | {cheapest})
            zz, _ = oracle.energy(n, edges, g, bt, threads=min(threads, len(sel)),
                                  edge_list=sel)
            rec.update(edge_ids=sel, energy=None)
        rec.update(zz_re=[float(z.real) for z in zz],
                   zz_im_max=float(max(abs(z.imag) for z in zz)),
                   oracle_width=[wmax[k] for k in rec["edge_ids"]],
                   oracle_seconds=round(time.time() - t0, 1))
        graphs.append(rec)
        print(f"graph {gi}: n={n} p={p} edges {len(rec['edge_ids'])}/{len(edges)} "
              f"width<={max(rec['oracle_width'])} {rec['oracle_seconds']} s", flush=True)
    out = {"case": "cfg3", **{k: (list(v) if isinstance(v, tuple) else v) for k, v in b.items()},
           "angle_set": 0, "graphs": graphs,
           "oracle": "FP64 bucket elimination, greedy min-fill per light cone",
           "oracle_seconds": round(time.time() - t_all, 1), "threads": threads}
    path = os.path.join(HERE, "cfg3_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(path, out["oracle_seconds"], "s")


if __name__ == "__main__":
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    if sys.argv[1] == "cfg3":
        make_batch(threads)
    else:
        make(sys.argv[1], threads)
