"""Writes the oracle's eigenvalues for the seeded workloads into tests/golden/.

Calls only the CPU oracle (oracle/) on inputs from the seeded generator; no
value here comes from the GPU path.  Each file records an input fingerprint
so a test can confirm it sees the same inputs.

    python tests/golden/make_golden.py workload2        # n = 1024, tall, ~25 min
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1907_08560_amd import synth  # noqa: E402


def fingerprint(P) -> list:
    return [float(np.abs(P.F).sum()), float(np.abs(P.G).sum()), int((P.J > 0).sum()),
            float(np.real(P.G[0, 0])), float(np.imag(P.F[-1, -1]))]


def run(name: str, P, reduce: bool):
    o = O.Oracle()
    t0 = time.time()
    st, lam, X, stats = o.ghsvd(P.F, P.J, P.G, reduce=reduce, order=0, max_sweeps=80)
    dt = time.time() - t0
    out = {"name": name, "status": int(st), "n": P.n, "m": P.m, "p": P.p, "reduce": reduce,
           "order": "row-cyclic", "max_sweeps": 80, "sweeps": int(stats[0]), "oracle_seconds": dt,
           "fingerprint": fingerprint(P), "lambda": [repr(float(v)) for v in lam]}
    with open(os.path.join(HERE, f"{name}_lambda.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(name, st, stats, f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    O.build()
    which = sys.argv[1:] or ["workload2"]
    for w in which:
        if w == "workload2":
            run("workload2", synth.workload_pencil(2), reduce=False)
        elif w == "workload1":
            run("workload1", synth.workload_pencil(1), reduce=False)
        else:
            raise SystemExit(f"unknown {w}")
