"""Writes the oracle's eigenvalues for the seeded workloads into tests/golden/.

Calls only the CPU oracle (oracle/) on inputs from the seeded generator; no
value here comes from the GPU path.  Each file records an input fingerprint
so a test can confirm it sees the same inputs.

    python tests/golden/make_golden.py workload2        # n = 1024, tall, ~7 min
    python tests/golden/make_golden.py workload4        # 64 pencils, a process pool
    python tests/golden/make_golden.py samples          # downsized workloads 3 and 5
    python tests/golden/make_golden.py parity           # uneven batch for the launch tests
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1907_08560_amd import synth  # noqa: E402


# orders of the uneven batch of the launch-configuration parity tests
PARITY_SIZES = [513, 257, 300, 130, 77]


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


def _one(job):
    """One pencil of a batch: (workload, k, n_override, j_identity) -> record.
    The oracle reduces the tall factors (Section 5) and sweeps the square ones
    in the round-robin order."""
    number, k, n_override, j_identity = job
    P = synth.workload_pencil(number, k, j_identity=j_identity, n_override=n_override)
    o = O.Oracle()
    t0 = time.process_time()
    st, lam, X, stats = o.ghsvd(P.F, P.J, P.G, reduce=True, order=1, max_sweeps=80)
    dt = time.process_time() - t0
    print(f"workload {number} pencil {k} n={P.n} status {st} sweeps {stats[0]} {dt:.1f}s",
          flush=True)
    # cancellation in h_j = f_j^* J f_j of each eigenvalue: kappa_j = ||F x_j||^2 / |lambda_j|
    # (>= 1; large for an eigenvalue near zero of an indefinite pencil)
    kap = np.sum(np.abs(P.F @ X) ** 2, axis=0) / np.abs(lam)
    return {"k": k, "status": int(st), "n": P.n, "m": P.m, "p": P.p, "m_plus": P.m_plus,
            "j_identity": j_identity, "sweeps": int(stats[0]), "oracle_cpu_seconds": dt,
            "fingerprint": fingerprint(P), "lambda": [repr(float(v)) for v in lam],
            "kappa_h": [float(f"{v:.3g}") for v in kap]}


def run_batch(name: str, jobs, desc: str):
    # largest pencils first, so the pool's tail is short
    order = sorted(jobs, key=lambda j: -(j[2] or synth.workload_sizes(j[0])[j[1]]))
    with mp.Pool(os.cpu_count() or 1) as pool:
        recs = pool.map(_one, order, chunksize=1)
    recs.sort(key=lambda r: r["k"])
    out = {"name": name, "description": desc, "reduce": True, "order": "round-robin",
           "max_sweeps": 80, "pencils": recs}
    with open(os.path.join(HERE, f"{name}_lambda.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    O.build()
    which = sys.argv[1:] or ["workload2"]
    for w in which:
        if w == "workload2":
            run("workload2", synth.workload_pencil(2), reduce=False)
        elif w == "workload1":
            run("workload1", synth.workload_pencil(1), reduce=False)
        elif w == "workload4":
            run_batch("workload4", [(4, k, None, False) for k in range(64)],
                      "all 64 pencils of workload 4 at full size")
        elif w == "samples":
            run_batch("workload5_sample", [(5, 0, 1000, False), (5, 1, 640, False)],
                      "pencils 0 and 1 of workload 5 (J 4:1, s in [1e-6, 1]) downsized "
                      "to n = 1000 and 640")
            run_batch("workload3_sample", [(3, 0, 1024, True), (3, 0, 768, False)],
                      "the workload-3 pencil (s in [1e-5, 1]) downsized to n = 1024 under "
                      "J = I, and to n = 768 with its 3:1 signature")
        elif w == "parity":
            run_batch("batch_parity", [(4, k, n, False) for k, n in enumerate(PARITY_SIZES)],
                      "pencils 0-4 of workload 4's recipe at n = " +
                      ", ".join(map(str, PARITY_SIZES)) + " (uneven orders across the 256- and "
                      "128-row Gram chunks, ragged last blocks and an empty padding block)")
        else:
            raise SystemExit(f"unknown {w}")
