#!/usr/bin/env python
"""QAOA MaxCut energy evaluations per second on one GPU.

Workload: random 3-regular graph, N=30 (45 edges, one light-cone network per
edge), QAOA depth p=4 -- the benchmark shape of Sec. II-E -- with seeded
angle sets gamma ~ U[0, pi), beta ~ U[0, pi/2).  One step evaluates
--angle-batch angle sets (default 32, all of them) in one pass over the plan:
angle upload, every bucket of every light cone for every set, the per-edge
scalars, the FP64 energies and their read-back; the reported value counts
every set's energy.  With --angle-batch 1 a step is one qtn_contract call on
one angle set.  The plan
(light cones, orders, merged groups, memory layout) is built once, before the
timed region, as a caller sweeping angles would.

Prints one JSON line.  `roofline` reports the dominant kernel class measured
with HIP events around each of its launches; `cpu_baseline` times the FP64
CPU oracle on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QAOA energy evals/s and bucket-contraction HBM GB/s, 3-reg N=30 p=4, 1 MI355X"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 (matrix / packed vector)
PAPER_SECONDS_PER_EVAL = 1.4  # Tab. II, NumPy_Merged + CuPy_Merged, V100 + CPU


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_tune(net, path):
    """Apply stored kernel choices (written by --save-tune on the same plan);
    None if the file is missing or was made for a different plan."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        stored = json.load(f)
    try:
        net.set_tune_picks(stored["picks"])
    except Exception as e:  # a different plan: tune afresh
        log(f"  stored tuning not applied ({e})")
        return None
    return {"source": os.path.relpath(path, ROOT), "n_groups": len(stored["picks"]),
            "measured_on": stored.get("measured_on")}


def save_tune(net, path, report, meta):
    with open(path, "w") as f:
        json.dump({**meta, "measured_on": "MI355X (gfx950)", "report": report,
                   "picks": [list(p) for p in net.tune_picks()]}, f)


def run_rows(Q, torch, inst, prec, levels, streams, steps, warmup, autotune=False,
             tune_file=None, save_tune_file=None, angle_batch=1, **cfg):
    """Plan (and tune) one network, then time `steps` steps after `warmup`.
    angle_batch 1: a step is one qtn_contract call on the next angle set;
    angle_batch K > 1: a step is one qtn_contract_angles call on K angle sets.
    Returns (network, seconds, plan seconds, last result, evaluations)."""
    n, edges = inst["n"], inst["edges"]
    angles = inst["angles"]
    net = Q.Network(n, edges, *angles[0], max_levels=levels, n_streams=streams, **cfg)
    t0 = time.perf_counter()
    net.plan(prec)
    plan_s = time.perf_counter() - t0
    ws = net.workspace()
    net.tune_report = None
    aws = None
    if angle_batch > 1:
        # one workspace for the angle batches and for tuning on them
        need = net.angles_workspace(angle_batch)
        if autotune:
            need = max(need, Q.qtn_tune_angles_workspace(net.h, angle_batch))
        aws = Q.workspace(need)
    if autotune:
        t0 = time.perf_counter()
        net.tune_report = load_tune(net, tune_file)
        if net.tune_report is None:
            # tuned on the workload that is timed: angle batches of this size
            net.tune_report = (net.autotune(aws, n_sets=angle_batch) if angle_batch > 1
                               else net.autotune(ws))
            if save_tune_file:
                save_tune(net, save_tune_file, dict(net.tune_report),
                          {"n": n, "edges": len(edges), "precision": prec, "levels": levels,
                           "angle_sets": angle_batch,
                           "config": {k: v for k, v in cfg.items() if k != "eager"}})
        net.tune_report["seconds"] = time.perf_counter() - t0
    if angle_batch > 1:
        import numpy as np
        sets = [angles[k % len(angles)] for k in range(angle_batch)]
        gs = np.array([a[0] for a in sets])
        bs = np.array([a[1] for a in sets])
        net.angle_sets = (gs, bs)
        net._aws = aws
        for _ in range(warmup):
            net.contract_angles(gs, bs, aws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for _ in range(steps):
            last = net.contract_angles(gs, bs, aws)
        torch.cuda.synchronize()
        return net, time.perf_counter() - t0, plan_s, last, steps * angle_batch
    for i in range(warmup):
        net.set_angles(*angles[i % len(angles)])
        net.contract(ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(steps):
        net.set_angles(*angles[(warmup + i) % len(angles)])
        last = net.contract(ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return net, dt, plan_s, last, steps


KERNEL_OF = {  # launch-log (kind, variant) -> kernel symbol
    (1, None): "k_block_groups", (2, 0): "k_wide_generic", (2, 1): "k_wide_stream",
    (2, 2): "k_wide_mfma", (2, 3): "k_wide_cells", (4, None): "k_persistent",
}


def kernel_name(rec):
    key = (rec["kind"], rec["variant"] if rec["kind"] == 2 else None)
    base = KERNEL_OF.get(key)
    if base is None:
        return None
    if rec["kind"] != 2:  # one instantiation serves every precision
        return base
    t = "double2" if rec["prec"] == 0 else "float2"
    cvt = 'true' if rec['cvt'] else 'false'
    if rec["variant"] == 3:  # one instantiation per cell and serial bit count
        return f"{base}<{t}, {cvt}, {rec['knob']}, {rec['serial']}>"
    if rec["variant"] == 2:  # one instantiation per column-block count
        return f"{base}<{t}, {cvt}, {rec['knob']}>"
    return f"{base}<{t}, {cvt}>"


def source_hash():
    """Hash of the kernel source, to tell whether stored counters still apply."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2204_06045_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, workload_tag):
    """Per-launch HBM bytes from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def roofline_of(log, workload_tag):
    """The kernel with the most device time in one timed evaluation, against
    its bound: algorithmic bytes (or flops) per launch over its mean launch
    duration (HIP events on the launch stream)."""
    per = {}
    for r in log:
        name = kernel_name(r)
        if name is None:
            continue
        a = per.setdefault(name, {"ms": 0.0, "bytes": 0.0, "flops": 0.0, "launches": 0,
                                  "c64_flops": 0.0})
        a["ms"] += r["ms"]
        if r["prec"] == 1:
            a["c64_flops"] += r["flops"]
        a["bytes"] += r["bytes"]
        a["flops"] += r["flops"]
        a["launches"] += 1
    kernel, t = max(per.items(), key=lambda kv: kv[1]["ms"])
    sec = t["ms"] / 1e3
    gbs = t["bytes"] / sec / 1e9 if sec > 0 else 0.0
    tflops = t["flops"] / sec / 1e12 if sec > 0 else 0.0
    # arithmetic peak of the precision the kernel's flops were done in
    fpeak = FP32_PEAK_TFLOPS if t["c64_flops"] >= 0.5 * t["flops"] else FP64_PEAK_TFLOPS
    hbm_frac, fp_frac = gbs / HBM_PEAK_GBS, tflops / fpeak
    n = max(1, t["launches"])
    common = {"kernel": kernel, "launches": t["launches"],
              "bytes_per_launch": t["bytes"] / n, "flops_per_launch": t["flops"] / n,
              "avg_launch_ms": t["ms"] / n, "hbm_gbs": gbs, "hbm_frac": hbm_frac,
              "fp_tflops": tflops, "fp_frac": fp_frac,
              "traffic": stored_traffic(kernel, workload_tag),
              "per_kernel": {k: {"ms": v["ms"], "launches": v["launches"],
                                 "gbs": v["bytes"] / max(v["ms"], 1e-9) / 1e6,
                                 "tflops": v["flops"] / max(v["ms"], 1e-9) / 1e9}
                             for k, v in per.items()}}
    if hbm_frac >= fp_frac:
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_frac, **common}
    return {"bound": "alu", "achieved": tflops, "peak": fpeak, "unit": "TFLOP/s",
            "frac": fp_frac, **common}


WIDTH_CLASSES = ((0, 12), (13, 17), (18, 23), (24, 64))


def launch_breakdown(log, n_sets=1):
    """Algorithmic GB/s of one timed evaluation (n_sets angle sets) per
    union-width class of the launches (a workgroup launch counts under its
    first group), the groups per second of the workgroup launches (the small
    buckets), and, for the matrix-form launches, the matrix cores' flops
    (3M: three real products, 6 * 2^w per group and angle set) against the matrix
    peak of their precision."""
    cls = {}
    for lo, hi in WIDTH_CLASSES:
        rs = [r for r in log if lo <= r["w"] <= hi]
        ms = sum(r["ms"] for r in rs)
        by = sum(r["bytes"] for r in rs)
        cls[f"w{lo}-{hi}"] = {"launches": len(rs), "ms": ms,
                              "gbs": by / ms / 1e6 if ms > 0 else 0.0}
    blk = [r for r in log if r["kind"] == 1]
    blk_ms = sum(r["ms"] for r in blk)
    mm = [r for r in log if r["kind"] == 2 and r["variant"] == 2]
    mm_ms = sum(r["ms"] for r in mm)
    # matrix-core work: 2^w complex multiply-adds per angle set, three real
    # products (3M, 6 real FLOPs) each, at the group's precision
    mm_flops = sum(6.0 * 2.0 ** r["w"] * n_sets for r in mm)
    mm_peak = (FP64_PEAK_TFLOPS if all(r["prec"] == 0 for r in mm) else FP32_PEAK_TFLOPS)
    # each launch against the bound its arithmetic intensity implies: the
    # time its bytes take at the HBM peak or its matrix work at the matrix
    # peak of its precision, whichever is longer
    bound_ms, n_hbm = 0.0, 0
    for r in mm:
        pk = FP64_PEAK_TFLOPS if r["prec"] == 0 else FP32_PEAK_TFLOPS
        t_hbm = r["bytes"] / (HBM_PEAK_GBS * 1e6)
        t_mm = 6.0 * 2.0 ** r["w"] * n_sets / (pk * 1e9)
        bound_ms += max(t_hbm, t_mm)
        n_hbm += t_hbm >= t_mm
    return {"width_classes": cls,
            "small_groups_per_s": (sum(r["n_groups"] for r in blk) / blk_ms * 1e3
                                   if blk_ms > 0 else 0.0),
            "matrix_form": ({"launches": len(mm), "ms": mm_ms,
                             "matrix_tflops": mm_flops / mm_ms / 1e9,
                             "peak_tflops": mm_peak,
                             "frac_matrix_peak": mm_flops / mm_ms / 1e9 / mm_peak,
                             "hbm_bound_launches": n_hbm,
                             "frac_of_bound": bound_ms / mm_ms}
                            if mm_ms > 0 else None)}


def golden_check(Q, net, inst, prec, last, angle_batch, seed):
    """Set 0 of the timed workload against the stored FP64 oracle values
    (tests/golden/cfg2_oracle.json: graph seed 0, angle set 0), outside the
    timed region.  Returns the comparison, or None when the workload is not
    the stored one; exits on a mismatch beyond the tolerance."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "cfg2_oracle.json")
    with open(path) as f:
        gd = json.load(f)
    g0, b0 = inst["angles"][0]
    if (seed != gd["seed"] or inst["n"] != gd["n"] or inst["p"] != gd["p"]
            or list(g0) != gd["gamma"] or list(b0) != gd["beta"]):
        return None
    if angle_batch > 1:
        zz, en = np.asarray(last[0])[0], float(np.asarray(last[1])[0])
    else:
        net.set_angles(g0, b0)
        zz, _, en = net.contract()
    tol = 1e-10 if prec == Q.QTN_C128 else 1e-5
    de = float(np.max(np.abs(np.asarray(zz) - np.asarray(gd["zz_re"]))))
    rel = abs(en - gd["energy"]) / abs(gd["energy"])
    out = {"angle_set": 0, "max_abs_delta_e": de, "energy_rel_err": rel, "tol": tol,
           "source": os.path.relpath(path, ROOT)}
    if not (de <= tol and rel <= tol):
        print(f"bench.py: set 0 differs from the FP64 oracle: {out}", file=sys.stderr)
        sys.exit(1)
    return out


def host_facts():
    """Logical CPUs and RAM of the host the oracle runs on."""
    try:
        ram = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES")
    except (ValueError, OSError, AttributeError):
        ram = None
    return {"logical_cpus": os.cpu_count(), "ram_bytes": ram}


def cpu_baseline(inst, threads=None):
    """One whole evaluation of the FP64 oracle on the host cores: every light
    cone of angle set 0, one oracle call per cone on a pool of host threads
    (heaviest cones first), timed as a whole (the multi-core rate) and cone
    by cone (the sum of the per-cone times is one core's time for the
    evaluation).  Nothing is sampled or scaled."""
    import concurrent.futures as cf

    import oracle
    n, edges, p = inst["n"], inst["edges"], inst["p"]
    g, b = inst["angles"][0]
    m = len(edges)
    threads = threads or max(1, min(os.cpu_count() or 1, 16))
    cost = [sum(2.0 ** int(w) for w in oracle.edge_widths(n, edges, k, p) if w) for k in range(m)]
    order = sorted(range(m), key=lambda k: -cost[k])

    def one(k):
        t0 = time.perf_counter()
        z, _ = oracle.energy(n, edges, g, b, threads=1, edge_list=[k])
        return k, z[0], time.perf_counter() - t0

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        done = list(ex.map(one, order))
    wall = time.perf_counter() - t0
    per_cone = sum(d[2] for d in done)
    energy = 0.5 * m - 0.5 * sum(d[1].real for d in done)
    return {"value": 1.0 / wall, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "value_1core": 1.0 / per_cone, "host": host_facts(), "energy": float(energy),
            "sample": (f"one whole evaluation: all {m} light cones of angle set 0, one "
                       f"single-threaded oracle call per cone on {threads} host threads, "
                       f"{wall:.1f} s wall; value_1core = 1 / the sum of the per-cone times "
                       f"({per_cone:.1f} s)")}


def batch_golden_check(insts, nets, zz, en, master_seed, count):
    """The last batched call's results against the stored FP64 oracle values
    (tests/golden/cfg3_oracle.json: every light cone of the graphs the oracle
    evaluated whole, the widest and the cheapest cones of the others),
    outside the timed region; exits on a mismatch beyond the complex64
    tolerance."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "cfg3_oracle.json")
    with open(path) as f:
        gd = json.load(f)
    if gd["master_seed"] != master_seed or gd["count"] != count:
        return None
    offs = np.cumsum([0] + [n.m for n in nets])
    de, rel, n_cones, n_en = 0.0, 0.0, 0, 0
    for rec in gd["graphs"]:
        i = rec["index"]
        it = insts[i]
        if (it["n"], it["p"], len(it["edges"])) != (rec["n"], rec["p"], rec["m"]):
            return None
        z = np.asarray(zz[offs[i]:offs[i + 1]])[np.asarray(rec["edge_ids"])]
        de = max(de, float(np.max(np.abs(z - np.asarray(rec["zz_re"])))))
        n_cones += len(rec["edge_ids"])
        if rec["energy"] is not None:
            rel = max(rel, abs(float(en[i]) - rec["energy"]) / abs(rec["energy"]))
            n_en += 1
    out = {"light_cones_compared": n_cones, "max_abs_delta_e": de, "energies_compared": n_en,
           "max_energy_rel_err": rel, "tol": 1e-5, "source": os.path.relpath(path, ROOT)}
    if not (de <= 1e-5 and rel <= 1e-5):
        print(f"bench.py: batched results differ from the FP64 oracle: {out}", file=sys.stderr)
        sys.exit(1)
    return out


def run_batch(Q, torch, steps, warmup, executor=5, autotune=False, order_trials=64,
              prec=1, master_seed=2204, count=64, slice_width=0, order_weight=4,
              hybrid_width=24, cost_model=None):
    """64 random cubic graphs, N uniform over even sizes in [20, 200], p in
    {2, 3, 4}; all light cones of all graphs in one batched call: the hybrid
    executor (cones up to width `hybrid_width` in one persistent lockstep
    launch, the wider ones by per-group launches after it), orders by the
    merged plan's flops + 4 x bytes.  With autotune: the 8 networks with the
    most algorithmic bytes are tuned, the trained cost model (cost_model)
    picks the kernels of the others, and the batched call's persistent grid
    and step item order are searched."""
    import qaoa_synth as qs
    insts = qs.batch_instances(master_seed, count, 20, 200, (2, 3, 4), d=3)
    t0 = time.perf_counter()
    nets = []
    for it in insts:
        g, b = it["angles"][0]
        net = Q.Network(it["n"], it["edges"], g, b, order_trials=order_trials,
                        executor=executor, slice_width=slice_width, order_weight=order_weight,
                        hybrid_width=hybrid_width)
        net.plan(prec)
        nets.append(net)
    plan_s = time.perf_counter() - t0
    tune_s = 0.0
    if autotune:
        # tune the 8 networks with the most algorithmic bytes (they carry most
        # of the batch's work; tuning all 64 would take minutes)
        t0 = time.perf_counter()
        heavy = sorted(nets, key=lambda n: -n.stats()["bytes"])[:8]
        for net in heavy:
            net.autotune()
        if cost_model is not None:
            for net in nets:
                if all(net is not h for h in heavy):
                    Q.qtn_apply_costmodel(net.h, cost_model)
        tune_s = time.perf_counter() - t0
        for net in nets:
            net._ws = None
        torch.cuda.empty_cache()
    handles = [n.h for n in nets]
    ws = Q.workspace(Q.qtn_batch_workspace(handles))
    total = sum(n.m for n in nets)
    sched_tune = None
    if autotune:
        # persistent grid and step item order of the batched call
        t0 = time.perf_counter()
        sched_tune = Q.qtn_autotune_batch(handles, ws)
        tune_s += time.perf_counter() - t0
    for _ in range(warmup):
        Q.qtn_contract_batch(handles, total, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        zz, en = Q.qtn_contract_batch(handles, total, ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    parity = batch_golden_check(insts, nets, zz, en, master_seed, count)
    st = [n.stats() for n in nets]
    row = {"graphs": count, "light_cones": total, "calls_per_s": steps / dt,
           "energies_per_s": count * steps / dt, "light_cones_per_s": total * steps / dt,
           "ms_per_call": 1e3 * dt / steps, "plan_seconds": plan_s, "tune_seconds": tune_s,
           "alg_bytes_per_call": sum(s["bytes"] for s in st),
           "max_width": max(s["max_width"] for s in st),
           "executor": {0: "persistent lockstep", 2: "persistent lockstep",
                        4: "persistent dataflow",
                        5: f"hybrid: persistent lockstep for cones up to width {hybrid_width}, "
                           "per-group launches for the wider ones"}.get(executor, "launches"),
           "kernel_choice": ("the 8 networks with the most bytes tuned, the others by the "
                             "learned cost model" if autotune and cost_model is not None else
                             "the 8 networks with the most bytes tuned, the others by the width "
                             "rule" if autotune else "width rule"),
           "precision": "c64" if prec == 1 else "c128", "order_trials": order_trials,
           "slice_width": slice_width, "order_weight": order_weight,
           "slices": sum(s["n_slices"] for s in st),
           "schedule_tune": sched_tune,
           "parity_vs_oracle": parity}
    for n in nets:
        n.close()
    return row


def run_seeds(Q, torch, seeds=(0, 1, 2, 3, 4), angle_batch=32, steps=6, order_trials=64,
              slice_width=0, order_weight=0):
    """The metric's shape on graph seeds 0-4 (the algorithmic bytes vary from
    graph to graph): per seed, the width of the widest bucket of each light
    cone (max and median), the histogram of bucket widths, the evaluation's
    algorithmic bytes, and evals/s of 32-set batches under the width rule (no
    tuning)."""
    import numpy as np
    import qaoa_synth as qs
    rows = {}
    for seed in seeds:
        inst = qs.instance(30, 3, 4, seed, angle_batch)
        g0, b0 = inst["angles"][0]
        net = Q.Network(30, inst["edges"], g0, b0, order_trials=order_trials,
                        slice_width=slice_width, order_weight=order_weight)
        net.plan(Q.QTN_C128)
        widths = [max(net.bucket_widths(e)) for e in range(len(inst["edges"]))]
        gs = np.array([a[0] for a in inst["angles"]])
        bs = np.array([a[1] for a in inst["angles"]])
        aws = Q.workspace(net.angles_workspace(angle_batch))
        for _ in range(2):
            net.contract_angles(gs, bs, aws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            net.contract_angles(gs, bs, aws)
        torch.cuda.synchronize()
        st = net.stats()
        rows[f"seed{seed}"] = {"evals_per_s": steps * angle_batch / (time.perf_counter() - t0),
                               "width_max": int(max(widths)),
                               "width_median": float(np.median(widths)),
                               # buckets per width (the planned light cones)
                               "width_hist": {str(w): int(c) for w, c in enumerate(st["width_hist"])
                                              if c},
                               "alg_bytes_per_eval": st["bytes"]}
        del aws
        net.close()
        torch.cuda.empty_cache()
    return rows


def run_gradient(Q, torch, inst, iters=12, lr=0.02, h=1e-4, order_trials=64, slice_width=0,
                 order_weight=0):
    """Parameter search on the metric's graph (Sec. II-A): gradient ascent on
    E(gamma, beta) with the gradient from one batched pass over 4p + 1 angle
    sets (qtn_energy_gradient), width rule, no tuning.  Reports gradients per
    second and the energy before and after."""
    import numpy as np
    g, b = (np.array(x, dtype=np.float64) for x in inst["angles"][0])
    net = Q.Network(inst["n"], inst["edges"], g, b, order_trials=order_trials,
                    slice_width=slice_width, order_weight=order_weight)
    net.plan(Q.QTN_C128)
    e0, dg, db = net.energy_gradient(g, b, step=h)  # warm-up (workspace, plan upload)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e = e0
    for _ in range(iters):
        e, dg, db = net.energy_gradient(g, b, step=h)
        g = g + lr * dg
        b = b + lr * db
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e_end, _, _ = net.energy_gradient(g, b, step=h)
    p = len(g)
    net.close()
    torch.cuda.empty_cache()
    return {"gradients_per_s": iters / dt, "energies_per_gradient": 4 * p + 1,
            "evals_per_s": iters * (4 * p + 1) / dt, "ascent_steps": iters,
            "learning_rate": lr, "step_h": h, "energy_start": e0, "energy_end": e_end}


def run_cfg4(Q, torch, steps=10, autotune=True, only=None):
    """4-regular N=40, p=3 (80 light cones): complex128, complex64 and mixed
    precision (groups of width >= 18 in complex64, in matrix form on the
    matrix cores where a group reshapes), each with its per-edge error
    against the stored FP64 oracle values; then complex128 and mixed with
    the headline's plan options (slicing at 26).  `only`: one row's name."""
    import numpy as np
    with open(os.path.join(ROOT, "tests", "golden", "cfg4_oracle.json")) as f:
        gd = json.load(f)
    ref = np.asarray(gd["zz_re"])
    rows = {}
    # the last two rows: the headline's plan options (best of 64 orders by
    # plan cost, slicing of cones wider than 26)
    for name, prec, variant, plan in (
            ("c128", Q.QTN_C128, 0, {}), ("c64", Q.QTN_C64, 0, {}),
            ("mixed", Q.QTN_MIXED, 0, {}), ("mixed_matrix", Q.QTN_MIXED, 3, {}),
            ("c128_sliced26", Q.QTN_C128, 0, dict(order_trials=64, slice_width=26, order_weight=4)),
            ("mixed_sliced26", Q.QTN_MIXED, 0,
             dict(order_trials=64, slice_width=26, order_weight=4))):
        if only is not None and name != only:
            continue
        net = Q.Network(gd["n"], gd["edges"], gd["gamma"], gd["beta"],
                        **{"order_trials": 16, "variant": variant, **plan})
        net.plan(prec)
        ws = net.workspace()
        if autotune:
            net.autotune(ws)
        zz, _, en = net.contract(ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            net.contract(ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        err = np.abs(zz - ref)
        st = net.stats()
        net.contract_timed(ws)
        mf = launch_breakdown(net.launch_log())["matrix_form"]
        rows[name] = {"evals_per_s": 1.0 / dt, "edge_err_max": float(err.max()),
                      "matrix_form": mf,
                      "edge_err_median": float(np.median(err)),
                      "energy_rel_err": abs(en - gd["energy"]) / abs(gd["energy"]),
                      "alg_bytes_per_eval": st["bytes"], "matrix_groups": st["n_matrix"],
                      "max_width": st["max_width"]}
        net.close()
        torch.cuda.empty_cache()
    return rows


def run_costmodel(Q, torch, prec=1, epochs=600, lr=3e-3, reps=3):
    """Train the cost model on autotuner timings of N=10 p=1, N=30 p=4 and 16
    of the batched graphs; evaluate it by measured time on 32 held-out graphs
    (16 cubic, 16 quartic, N even in [50, 500], p=3) against the width rule."""
    import numpy as np
    import qaoa_synth as qs
    feats, times = [], []

    def collect(n, edges, g, b, trials):
        net = Q.Network(n, edges, g, b, order_trials=trials)
        net.plan(prec)
        net.autotune()
        f, m = net.tune_log()
        feats.append(f)
        times.append(m)
        net.close()

    t0 = time.perf_counter()
    for seed in range(3):
        it = qs.instance(10, 3, 1, seed)
        collect(10, it["edges"], *it["angles"][0], 0)
    it = qs.instance(30, 3, 4, 0)
    collect(30, it["edges"], *it["angles"][0], 64)
    for it in qs.batch_instances(2204, 64, 20, 200, (2, 3, 4), d=3)[:16]:
        collect(it["n"], it["edges"], *it["angles"][0], 16)
    x = np.concatenate(feats)
    ms = np.concatenate(times)
    collect_s = time.perf_counter() - t0
    r = qs.Rng(4242)
    init = np.array([0.15 * (2 * r.uniform() - 1) for _ in range(Q.CostModel.n_params)],
                    dtype=np.float32)
    cm = Q.CostModel(init)
    t0 = time.perf_counter()
    hist = cm.train(x, ms, epochs, lr)
    train_s = time.perf_counter() - t0
    torch.cuda.empty_cache()
    rr = qs.Rng(5000)
    fallback_ms = learned_ms = 0.0
    gains = []
    picks = np.zeros(4, dtype=np.int64)
    for i in range(32):
        d = 3 if i < 16 else 4
        sizes = [n for n in range(50, 501) if (n * d) % 2 == 0]
        n = sizes[rr.below(len(sizes))]
        inst = qs.instance(n, d, 3, 7000 + i)
        # the same plan twice: width rule, and the model's picks; timed in
        # alternation so that drift hits both alike
        fb = Q.Network(n, inst["edges"], *inst["angles"][0], order_trials=4)
        fb.plan(prec)
        ln = Q.Network(n, inst["edges"], *inst["angles"][0], order_trials=4)
        ln.plan(prec)
        picks += Q.qtn_apply_costmodel(ln.h, cm)
        wf, wl = fb.workspace(), ln.workspace()
        fb.contract(wf)
        ln.contract(wl)
        tf = tl = 0.0
        for _ in range(reps):
            for net, ws in ((fb, wf), (ln, wl)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                net.contract(ws)
                torch.cuda.synchronize()
                dt = 1e3 * (time.perf_counter() - t0)
                if net is fb:
                    tf += dt
                else:
                    tl += dt
        fallback_ms += tf / reps
        learned_ms += tl / reps
        gains.append(tf / tl)
        fb.close()
        ln.close()
        torch.cuda.empty_cache()
    return {"train_samples": int(len(x)), "collect_seconds": collect_s,
            "train_seconds": train_s, "epochs": epochs, "loss_first": float(hist[0]),
            "loss_last": float(hist[-1]), "heldout_graphs": 32,
            "fallback_ms_per_pass": fallback_ms, "learned_ms_per_pass": learned_ms,
            "gain": fallback_ms / learned_ms if learned_ms > 0 else None,
            "gain_per_graph": {"min": float(min(gains)), "median": float(np.median(gains)),
                               "max": float(max(gains))},
            "picks_block_stream_generic_mfma": [int(v) for v in picks],
            "precision": "c64" if prec == 1 else "c128",
            "_model": cm}


def run_micro(Q, torch, reps=5, n_random=8, seed=2204):
    """Single-bucket probes of the bucket kernels (Sec. II-E synthetic
    benchmarks, Tab. III), each one bucket of binary indices on the network
    path's kernels (qtn_bucket_*): matrix products (k summed labels), the
    fixed abcd,bcdf->acf contraction (each index 2^4 as 4 labels) and random
    two-operand contractions of 16..25 distinct labels with 1..8 summed.
    Kernel time from events attached to the dispatch, the median of `reps`
    runs after one warm-up; inputs seeded normal values.  Each row carries
    algorithmic GB/s, true and paper-convention (8 * 2^labels) flop rates and
    the fraction of the roof its arithmetic intensity implies."""
    import numpy as np
    import qaoa_synth as qs

    def probe(ops, out, prec, variant=0):
        b = Q.Bucket(ops, out, precision=prec, variant=variant)
        info = b.info()
        data = torch.empty(info["data_bytes"], dtype=torch.uint8, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        data.view(torch.float64 if prec == Q.QTN_C128 else torch.float32).normal_(generator=g)
        b.contract_timed(data)
        ms = float(np.median([b.contract_timed(data) for _ in range(reps)]))
        b.close()
        del data
        gbs = info["bytes"] / ms / 1e6
        tflops = info["flops"] / ms / 1e9
        # FP64 (complex128) or FP32 (complex64) arithmetic: the vector ALUs,
        # or in matrix form the matrix cores of the same precision, whose
        # work is three real products (3M, 6 real FLOPs) per union point
        fpeak = FP64_PEAK_TFLOPS if prec == Q.QTN_C128 else FP32_PEAK_TFLOPS
        row = {"w": info["w"], "L": info["L"], "mapping": ["generic", "streaming", "matrix form",
                                                           "cells"][info["variant"]],
               "kernel_ms": ms, "gbs": gbs, "tflops": tflops,
               "paper_gflops": 8.0 * 2.0 ** info["w"] / ms / 1e6}
        if info["variant"] == 2:
            # against the bound its intensity implies (3M matrix work vs bytes)
            mt = 6.0 * 2.0 ** info["w"] / ms / 1e9
            hbm = 6.0 * 2.0 ** info["w"] / info["bytes"] < fpeak * 1e12 / (HBM_PEAK_GBS * 1e9)
            return {**row, "matrix_tflops": mt, "bound": "hbm" if hbm else "mfma",
                    "frac": gbs / HBM_PEAK_GBS if hbm else mt / fpeak}
        bound = "hbm" if info["flops"] / info["bytes"] < fpeak * 1e12 / (HBM_PEAK_GBS * 1e9) else "alu"
        frac = gbs / HBM_PEAK_GBS if bound == "hbm" else tflops / fpeak
        return {**row, "bound": bound, "frac": frac}

    rows = {}
    for name, prec in (("c128", Q.QTN_C128), ("c64", Q.QTN_C64)):
        k = list(range(8))
        for mb, nb in ((8, 8), (11, 12)):
            m_ = list(range(8, 8 + mb))
            n_ = list(range(8 + mb, 8 + mb + nb))
            shape = f"{1 << mb}x{1 << nb}x256"
            rows[f"matmul_{shape}_{name}"] = probe([k + m_, k + n_], m_ + n_, prec)
            rows[f"matmul_{shape}_{name}_matrix_form"] = probe([k + m_, k + n_], m_ + n_, prec,
                                                                variant=3)
        a, bb, c, d, f = ([4 * i + j for j in range(4)] for i in range(5))
        rows[f"tncontract_fixed_n16_{name}"] = probe([bb + d + a + c, bb + d + c + f], a + c + f, prec)
        r = qs.Rng(seed)
        rnd = []
        for _ in range(n_random):
            n_lab = 16 + r.below(10)
            n_sum = 1 + r.below(8)
            summed = list(range(n_sum))
            kept = list(range(n_sum, n_lab))
            # each kept label in one operand or both; every summed label in both
            side = [r.below(3) for _ in kept]
            A = summed + [l for l, sd in zip(kept, side) if sd != 1]
            B = summed + [l for l, sd in zip(kept, side) if sd != 0]
            rnd.append(probe([A, B], kept, prec))
        rows[f"tncontract_random_{name}"] = {
            "cases": n_random, "labels": [x["w"] for x in rnd],
            "median_gbs": float(np.median([x["gbs"] for x in rnd])),
            "median_frac": float(np.median([x["frac"] for x in rnd])),
            "median_paper_gflops": float(np.median([x["paper_gflops"] for x in rnd])),
            "rows": rnd}
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=("c128", "c64", "mixed"), default="c128")
    ap.add_argument("--mixed-width", type=int, default=0,
                    help="mixed: narrowest group run in complex64 (0 = library default)")
    ap.add_argument("--levels", type=int, default=8, help="merged indices per group (1 = plain)")
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--small-width", type=int, default=0, help="widest group run in-block")
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 generic, 2 streaming")
    ap.add_argument("--lane-bits", type=int, default=0, help="streaming lane-summed bits")
    ap.add_argument("--executor", type=int, default=0, help="0 default, 1 launches, 2 persistent")
    ap.add_argument("--order-trials", type=int, default=64,
                    help="randomized min-fill orders tried per light cone (0 = greedy)")
    ap.add_argument("--order-weight", type=int, default=4,
                    help="order search by plan flops + this weight * bytes (0: sum of 2^width)")
    ap.add_argument("--slice-width", type=int, default=24,
                    help="index slicing of light cones wider than this (0: off)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--angle-sets", type=int, default=32)
    ap.add_argument("--angle-batch", type=int, default=32,
                    help="angle sets evaluated per step in one pass (1: one call per set)")
    ap.add_argument("--variants", type=int, default=1, help="also time the other rows")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the oracle baseline (0: all, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=1,
                    help="tune the kernel choice per group after planning (stored choices "
                         "from --tune-file when they match the plan, else the autotuner)")
    ap.add_argument("--tune-file", default=None,
                    help="stored kernel choices to apply (default: paper_2204_06045_amd/tuning/tune_n30p4_<prec>.json)")
    ap.add_argument("--retune", action="store_true", help="ignore stored choices, measure afresh")
    ap.add_argument("--save-tune", default=None, help="write the autotuner's choices here")
    ap.add_argument("--eager", action="store_true",
                    help="launch eagerly instead of replaying the captured HIP graph")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (byte-counter calibration)")
    ap.add_argument("--cfg4", nargs="?", const="all", default=None,
                    choices=("all", "c128", "c64", "mixed", "mixed_matrix", "c128_sliced26",
                             "mixed_sliced26"),
                    help="only the 4-regular N=40 p=3 rows (or one of them): one JSON line")
    ap.add_argument("--micro", action="store_true",
                    help="only the single-bucket probes (matrix products, fixed and random "
                         "contractions): one JSON line of their rows")
    ap.add_argument("--batch", action="store_true",
                    help="only the 64-graph batch row (hybrid executor; with --autotune 0 "
                         "every kernel by the width rule): one JSON line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(light cones shard across GPUs without communication; only the "
              "one-GPU share is built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2204_06045_amd as Q
    import qaoa_synth as qs

    torch.cuda.set_device(0)
    if args.micro:
        print(json.dumps({"micro": run_micro(Q, torch)}))
        return
    if args.batch:
        print(json.dumps({"batch64_c64": run_batch(Q, torch, max(1, args.steps // 8),
                                                   min(args.warmup, 2),
                                                   autotune=bool(args.autotune))}))
        return
    if args.cfg4:
        print(json.dumps({"n40d4p3": run_cfg4(Q, torch, autotune=bool(args.autotune),
                                              only=None if args.cfg4 == "all" else args.cfg4)}))
        return
    inst = qs.instance(30, 3, 4, args.seed, args.angle_sets)
    prec = {"c128": Q.QTN_C128, "c64": Q.QTN_C64, "mixed": Q.QTN_MIXED}[args.precision]
    log(f"main row: {args.precision} levels={args.levels} streams={args.streams}")
    kcfg = dict(variant=args.variant, lane_sum_bits=args.lane_bits,
                order_trials=args.order_trials, executor=args.executor,
                small_width=args.small_width, mixed_width=args.mixed_width, eager=args.eager,
                slice_width=args.slice_width, order_weight=args.order_weight)
    tag_s = ((f"_s{args.slice_width}" if args.slice_width else "") +
             (f"_o{args.order_weight}" if args.order_weight else ""))
    tune_file = None if args.retune else (
        args.tune_file or os.path.join(ROOT, "paper_2204_06045_amd", "tuning",
                                       f"tune_n30p4_{args.precision}{tag_s}.json"))
    net, dt, plan_s, last, n_evals = run_rows(
        Q, torch, inst, prec, args.levels, args.streams, args.steps, args.warmup,
        autotune=bool(args.autotune), tune_file=tune_file, save_tune_file=args.save_tune,
        angle_batch=args.angle_batch, **kcfg)
    tune = net.tune_report
    evals = n_evals / dt
    parity = golden_check(Q, net, inst, prec, last, args.angle_batch, args.seed)
    if parity is not None:
        log(f"  set 0 vs FP64 oracle: max |delta e| {parity['max_abs_delta_e']:.2e}, "
            f"|delta E|/E {parity['energy_rel_err']:.2e}")
    stats = net.stats()
    log(f"  {evals:.2f} evals/s ({args.angle_batch} angle sets per step), plan {plan_s:.2f} s")
    # kernel roofline: the same tuned plan and step, its launches serialized
    # on one stream so that each launch's HIP event pair brackets that kernel
    if args.angle_batch > 1:
        gs, bs = net.angle_sets
        net.contract_angles(gs, bs, timed=True)
        _, _, timing = net.contract_angles(gs, bs, timed=True)
    else:
        net.contract_timed()
        _, _, timing = net.contract_timed()
    tag = (f"n30p4_{args.precision}{tag_s}" +
           (f"_x{args.angle_batch}" if args.angle_batch > 1 else ""))
    main_log = net.launch_log()
    roof = roofline_of(main_log, tag)
    breakdown = launch_breakdown(main_log, args.angle_batch)
    # the same plan, one qtn_contract call per angle set
    sequential = None
    if args.angle_batch > 1 and args.variants:
        ws1 = net.workspace()
        for i in range(3):
            net.set_angles(*inst["angles"][i % len(inst["angles"])])
            net.contract(ws1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.angle_batch):
            net.set_angles(*inst["angles"][i % len(inst["angles"])])
            net.contract(ws1)
        torch.cuda.synchronize()
        sequential = {"evals_per_s": args.angle_batch / (time.perf_counter() - t0),
                      "note": "same plan and kernels, one qtn_contract call per angle set"}
    net.close()
    log(f"  roofline {roof['kernel']}: {roof['hbm_gbs']:.0f} GB/s, "
        f"{roof['fp_tflops']:.2f} TFLOP/s")
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    variants = {}
    if sequential is not None:
        variants[f"sequential_{args.precision}"] = sequential
    if args.variants:
        # merged rows with the main row's angle batch (and its slicing and
        # order objective); the merged plan with neither (orders by the sum
        # of 2^width, no slicing; its stored kernel choices); the
        # bucket-by-bucket rows (the plain per-bucket path: no merging, no
        # slicing) one call per angle set, as the paper's backends run
        ow = args.order_weight
        for name, pr, lv, ab, sw, vw in (
                ("c128_merged", Q.QTN_C128, 8, args.angle_batch, args.slice_width, ow),
                ("c128_unsliced", Q.QTN_C128, 8, args.angle_batch, 0, 0),
                ("c64_merged", Q.QTN_C64, 8, args.angle_batch, args.slice_width, ow),
                ("mixed_merged", Q.QTN_MIXED, 8, args.angle_batch, args.slice_width, ow),
                ("c128_plain", Q.QTN_C128, 1, 1, 0, 0), ("c64_plain", Q.QTN_C64, 1, 1, 0, 0)):
            if (pr == prec and lv == args.levels and ab == args.angle_batch
                    and sw == args.slice_width and vw == ow):
                continue
            log(f"variant {name}")
            vsteps = max(3, args.steps // 4) if ab == 1 else max(2, args.steps // 8)
            vtune = None
            if sw == 0 and vw == 0 and lv == 8 and pr == Q.QTN_C128 and not args.retune:
                vtune = os.path.join(ROOT, "paper_2204_06045_amd", "tuning", "tune_n30p4_c128.json")
            vnet, vdt, _, _, vev = run_rows(Q, torch, inst, pr, lv, args.streams, vsteps, 2,
                                            autotune=bool(args.autotune), tune_file=vtune,
                                            angle_batch=ab,
                                            **{**kcfg, "slice_width": sw, "order_weight": vw})
            vst = vnet.stats()
            variants[name] = {"evals_per_s": vev / vdt, "angle_sets_per_step": ab,
                              "alg_bytes_per_eval": vst["bytes"],
                              "alg_flops_per_eval": vst["flops"], "slice_width": sw,
                              "order_weight": vw,
                              "slices": vst["n_slices"], "n_groups": vst["n_groups"]}
            vnet.close()
            torch.cuda.empty_cache()

    if args.variants:
        log("variant cfg4 (4-regular N=40 p=3: c128, c64, mixed, mixed + matrix form)")
        variants["n40d4p3"] = run_cfg4(Q, torch, autotune=bool(args.autotune))
        torch.cuda.empty_cache()
        log("variant costmodel (learned selector vs width rule, held-out graphs)")
        variants["costmodel_c64"] = run_costmodel(Q, torch)
        cost_model = variants["costmodel_c64"].pop("_model")
        torch.cuda.empty_cache()
        log("variant gradient (gradient ascent, 4p + 1 angle sets per gradient)")
        variants["gradient_c128"] = run_gradient(Q, torch, inst, slice_width=args.slice_width,
                                                 order_weight=args.order_weight)
        torch.cuda.empty_cache()
        log("variant seeds (graph seeds 0-4, width rule, 32-set batches)")
        variants["seeds_c128"] = run_seeds(Q, torch, slice_width=args.slice_width,
                                           order_weight=args.order_weight)
        torch.cuda.empty_cache()
        log("variant micro (single-bucket probes)")
        variants["micro"] = run_micro(Q, torch)
        torch.cuda.empty_cache()
        log("variant batch64_c64 (hybrid executor)")
        variants["batch64_c64"] = run_batch(Q, torch, 5, 1, autotune=bool(args.autotune),
                                            cost_model=cost_model)
        cost_model.close()
        torch.cuda.empty_cache()
        log("variant batch64_c64_lockstep (every cone in the persistent lockstep launch)")
        variants["batch64_c64_lockstep"] = run_batch(Q, torch, 5, 1, executor=0, order_trials=16,
                                                     order_weight=0, autotune=False)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(inst, args.cpu_threads or None)

    line = {
        "metric": METRIC,
        "value": evals,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": evals * PAPER_SECONDS_PER_EVAL,
        "vs_baseline_note": ("paper Tab. II best: 1.4 s per evaluation (NumPy_Merged + "
                             "CuPy_Merged, V100 + host CPU, its own graph instance); context"),
        "dtype": {0: "complex128", 1: "complex64", 2: "complex128+complex64"}[prec],
        "data": "synthetic",
        "config": {
            "workload": (f"QAOA MaxCut energy, random 3-regular N=30 (45 edges), p=4, graph "
                         f"seed {args.seed}, {args.angle_sets} seeded angle sets"),
            "precision": args.precision, "max_levels": args.levels,
            "streams": args.streams, "variant": args.variant,
            "lane_sum_bits": args.lane_bits, "order_trials": args.order_trials,
            "executor": args.executor, "autotune": bool(args.autotune), "eager": args.eager,
            "slice_width": args.slice_width, "order_weight": args.order_weight,
            "angle_sets_per_step": args.angle_batch,
            "max_width": stats["max_width"],
            "buckets": stats["n_buckets"], "groups": stats["n_groups"],
        },
        "alg_bytes_per_eval": stats["bytes"],
        "alg_flops_per_eval": stats["flops"],
        "eval_hbm_gbs": stats["bytes"] * evals / 1e9,
        "paper_gflops_per_s": stats["paper_flops"] * evals / 1e9,
        "launch_breakdown": breakdown,
        "plan_seconds": plan_s,
        "autotune": tune,
        "roofline": roof,
        "parity_vs_oracle": parity,
        "kernel_timing": timing,
        "kernel_source_hash": source_hash(),
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
