"""Write the FP64-oracle expected values used by the full-size GPU parity tests.

Calls only ``oracle/`` (bucket elimination with its own min-fill orders, in
double complex) on seeded synthetic instances from ``qaoa_synth``; no value
comes from the HIP library.

    python tests/golden/make_golden.py cfg2 [threads]
"""

from __future__ import annotations

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


if __name__ == "__main__":
    make(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 4)
