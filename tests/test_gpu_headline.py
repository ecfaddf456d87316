"""Parity in the launch configuration the benchmark's headline times: batched
blocked solves (mixed FP32 warm-up + FP64 finish, and plain FP64) with the
tuner's widths (w = 16 and 32, 8 wavefronts per pair), against the oracle's
eigenvalues stored in tests/golden/ (written by make_golden.py, which calls
only the CPU oracle: its reduction of the tall factors, then round-robin
sweeps on the square ones).

Inputs:
  * an uneven batch from the 64-pencil recipe at n = 513, 257, 300, 130, 77
    (ragged last blocks, an empty padding block, Gram chunks of 256 and 128
    rows cut at different places);
  * the full 64-pencil batch (n_k in [300, 900]);
  * the large-pencil recipe (J 4:1, s in [1e-6, 1]) downsized to n = 1000
    and 640, and the n = 4096 recipe (s in [1e-5, 1]) downsized to n = 1024
    under J = I and to n = 768 with its 3:1 signature.

Tolerance: cond(S) <= 1e12 in all of them, where the per-eigenvalue relative
error of the method is about 0.05 eps kappa(G) <= 1e-11 on either side; the
gate is 1e-10.  An eigenvalue near zero of the indefinite pencil is also
sensitive to the cancellation in h_j = f_j^* J f_j: with kappa_j = ||F x_j||^2
/ |lambda_j| (stored beside the oracle's eigenvalues), rounding errors of
relative size eps in the columns of F -- the hyperbolic reflectors of the
reduction and the rotations of the sweeps each add one, so about sqrt(m n)
of them accumulate in a column as a random walk -- move lambda_j by about
sqrt(m n) eps kappa_j relative, on each side.  The gate per eigenvalue is
1e-10 + 4 sqrt(m n) eps kappa_j (for kappa_j <= 100 the second term is below
1e-11).  The count of negative eigenvalues (the inertia of H) must agree
exactly, and a batched pencil must equal its own single solve bit for bit
(no reduction crosses pencils).
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, to_dev

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10


def fingerprint(P):
    return [float(np.abs(P.F).sum()), float(np.abs(P.G).sum()), int((P.J > 0).sum()),
            float(np.real(P.G[0, 0])), float(np.imag(P.F[-1, -1]))]


EPS = 2.0 ** -52


def load(name, make):
    """Golden records of a batch and the matching seeded pencils: (pencils,
    list of (oracle eigenvalues, per-eigenvalue tolerance))."""
    g = json.load(open(os.path.join(HERE, "golden", f"{name}_lambda.json")))
    Ps, refs = [], []
    for r in g["pencils"]:
        P = make(r)
        assert np.allclose(fingerprint(P), r["fingerprint"], rtol=1e-12, atol=0), "generator drift"
        assert r["status"] == 0
        Ps.append(P)
        lam = np.array([float(v) for v in r["lambda"]])
        kap = np.asarray(r.get("kappa_h", np.ones_like(lam)), dtype=np.float64)
        refs.append((lam, TOL + 4.0 * np.sqrt(float(P.m) * P.n) * EPS * kap))
    return Ps, refs


def check(lams, refs, tag):
    worst = worst_ratio = 0.0
    for k, (lam, (ref, tol)) in enumerate(zip(lams, refs)):
        lam = host(lam)
        rel = np.abs(lam - ref) / np.abs(ref)
        worst = max(worst, float(rel.max()))
        worst_ratio = max(worst_ratio, float((rel / tol).max()))
        j = int(np.argmax(rel / tol))
        assert rel[j] <= tol[j], (tag, k, j, float(ref[j]), float(rel[j]), float(tol[j]))
        assert int((lam < 0).sum()) == int((ref < 0).sum()), (tag, k)
    print(f"{tag}: worst rel err {worst:.2e}, worst err / gate {worst_ratio:.2f} over "
          f"{len(refs)} pencils", flush=True)


@pytest.fixture(scope="module")
def parity_batch():
    return load("batch_parity", lambda r: synth.workload_pencil(4, r["k"], n_override=r["n"]))


@pytest.mark.parametrize("w", [16, 32])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_uneven_batch_matches_oracle(parity_batch, w, precision):
    Ps, refs = parity_batch
    dev = [to_dev(P) for P in Ps]
    kw = dict(precision=precision, variant="blocked", block_width=w, waves_per_pair=8)
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], **kw)
    assert rc == 0, [i["status"] for i in infos]
    check(lams, refs, f"uneven batch {precision} w={w}")
    for k in (0, 4):
        lam1, X1, info1 = ghsvd.solve(*dev[k], **kw)
        assert torch.equal(lam1, lams[k]) and torch.equal(X1, Xs[k]), k


@pytest.fixture(scope="module")
def workload4():
    return load("workload4", lambda r: synth.workload_pencil(4, r["k"]))


@pytest.mark.parametrize("precision,w", [("mixed", 16), ("mixed", 32), ("fp64", 16)])
def test_workload4_full_batch(workload4, precision, w):
    Ps, refs = workload4
    assert len(Ps) == 64
    dev = [to_dev(P) for P in Ps]
    lams, Xs, infos, rc = ghsvd.solve_batched([d[0] for d in dev], [d[1] for d in dev],
                                              [d[2] for d in dev], precision=precision,
                                              variant="blocked", block_width=w, waves_per_pair=8)
    assert rc == 0, [i["status"] for i in infos]
    check(lams, refs, f"workload 4 {precision} w={w}")


def test_large_pencil_samples():
    Ps5, refs5 = load("workload5_sample",
                      lambda r: synth.workload_pencil(5, r["k"], n_override=r["n"]))
    Ps3, refs3 = load("workload3_sample",
                      lambda r: synth.workload_pencil(3, r["k"], n_override=r["n"],
                                                      j_identity=r["j_identity"]))
    assert Ps3[0].m_plus == Ps3[0].m or Ps3[1].m_plus == Ps3[1].m  # one J = I pencil
    for tag, Ps, refs in (("large-pencil sample", Ps5, refs5), ("n=4096 sample", Ps3, refs3)):
        dev = [to_dev(P) for P in Ps]
        for precision in ("mixed", "fp64"):
            lams, Xs, infos, rc = ghsvd.solve_batched(
                [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev],
                precision=precision, variant="blocked")
            assert rc == 0, [i["status"] for i in infos]
            check(lams, refs, f"{tag} {precision}")
