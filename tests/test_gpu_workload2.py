"""The n = 1024 workload at full size (F 1536 x 1024, G 2048 x 1024,
cond(S) = 1e16) in the launch configuration the benchmark times, against the
oracle's eigenvalues stored in tests/golden/ (written by make_golden.py, which
calls only the CPU oracle: tall factors, row-cyclic Algorithm 2).

Tolerance: at cond(S) = 1e16 (kappa(G) = 1e8) the per-eigenvalue error of the
method itself is about 0.05 eps kappa(G) ~ 1e-9 (the oracle against 40-digit
brute force at this conditioning shows 0.7e-9 .. 1.3e-9 as its worst), so GPU
and oracle may differ by a few times that: the gate is 1e-8 (measured 2.7e-9
on every path).  The median error is also reported.
"""
import json
import os

import numpy as np
import pytest

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import factor_invariants, host, to_dev

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pencil():
    P = synth.workload_pencil(2)
    g = json.load(open(os.path.join(HERE, "golden", "workload2_lambda.json")))
    fp = [float(np.abs(P.F).sum()), float(np.abs(P.G).sum()), int((P.J > 0).sum()),
          float(np.real(P.G[0, 0])), float(np.imag(P.F[-1, -1]))]
    assert np.allclose(fp, g["fingerprint"], rtol=1e-12, atol=0), "generator drift"
    lam_o = np.array([float(v) for v in g["lambda"]])
    return P, lam_o


@pytest.mark.parametrize("precision,variant", [("fp64", "pointwise"), ("fp64", "blocked"),
                                               ("mixed", "blocked"), ("mixed", "pointwise")])
def test_workload2_full_size(pencil, precision, variant):
    P, lam_o = pencil
    F, J, G = to_dev(P)
    lam, X, info = ghsvd.solve(F, J, G, precision=precision, variant=variant)
    assert info["status"] == 0, info
    lam = host(lam)
    rel = np.abs(lam - lam_o) / np.abs(lam_o)
    print(f"{precision}/{variant}: max rel err {rel.max():.3e} median {np.median(rel):.3e} "
          f"sweeps fp32 {info['sweeps_fp32']} fp64 {info['sweeps_fp64']} "
          f"blocked {info['sweeps_blocked']}", flush=True)
    assert rel.max() <= 1e-8
    assert np.median(rel) <= 1e-11
    # same count of negative eigenvalues (the inertia of H)
    assert int((lam < 0).sum()) == int((lam_o < 0).sum())
    # sampled invariants on the factors (64 columns)
    idx = np.linspace(0, P.n - 1, 64).astype(int)
    Xs = host(X)[:, idx]
    GX = P.G @ Xs
    assert np.abs(GX.conj().T @ GX - np.eye(len(idx))).max() < 1e-6
