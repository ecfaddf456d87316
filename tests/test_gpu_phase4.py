"""GPU parity of the full GHSVD from swept factors (ghsvd_full; Phase 4,
Section 7, with the outputs of Section 6.1) against the oracle.

sigma_f, sigma_g, U and V are plain scalings and are compared element by
element; X = Z^{-1} is unique, so it is compared element by element within
eps times the condition number of Z (the pivot sequences of the two
complete-pivoting factorizations may differ where moduli nearly tie, and are
not compared).
"""
import numpy as np
import pytest
import torch

from oracle import phase4
from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host

pytestmark = pytest.mark.gpu


def dev(a):
    return ghsvd.to_device_fortran(np.asarray(a, dtype=np.complex128))


@pytest.mark.parametrize("number,n_override", [(1, None), (2, 100), (4, 130)])
def test_full_matches_oracle(oracle, number, n_override):
    P = synth.workload_pencil(number, n_override=n_override)
    st, Fp, Gp, Zp, _ = oracle.hz_run(P.F, P.J, P.G, max_sweeps=60)
    assert st == 0
    U, V, sf, sg, X = ghsvd.full(dev(Fp), P.m_plus, dev(Gp), dev(Zp))
    Uo, Vo, sfo, sgo, Xo = phase4.full_ghsvd(Fp, P.J, Gp, Zp)
    assert np.abs(host(sf) - sfo).max() <= 1e-14
    assert np.abs(host(sg) - sgo).max() <= 1e-14
    for A, B in ((host(U), Uo), (host(V), Vo)):
        assert np.max(np.abs(A - B) / np.linalg.norm(B, axis=0)[None, :]) < 1e-13
    Z = Zp / np.sqrt((np.abs(np.sum(np.conj(Fp) * (P.J[:, None] * Fp), axis=0))
                      + np.sum(np.abs(Gp) ** 2, axis=0)))[None, :]
    kz = np.linalg.cond(Z)
    Xh = host(X)
    assert np.abs(Xh - Xo).max() <= 1e-14 * kz * np.abs(Xo).max(), (np.abs(Xh - Xo).max(), kz)
    assert np.abs(Xh @ Z - np.eye(P.n)).max() <= 1e-14 * kz * P.n
    # the relative errors (7.1) of the decomposition of the starting factors
    eF, eG = phase4.decomposition_errors(P.F, P.G, host(U), host(V), host(sf), host(sg), Xh)
    assert eF < 1e-12 and eG < 1e-12, (eF, eG)


def test_full_after_gpu_reduction_and_blocked_sweeps(oracle):
    # the whole GPU path: reduction, row split by the signature, blocked
    # sweeps in place, then the full GHSVD of the square factors
    P = synth.random_pencil(321, 256, 384, 288, 512, 1e-3)
    F = dev(P.F)
    G = dev(P.G)
    J = torch.from_numpy(P.J).cuda()
    Fsq, Jsq, Gsq, perm, n2 = ghsvd.reduce(F, J, G)
    js = host(Jsq)
    order = np.concatenate([np.flatnonzero(js > 0), np.flatnonzero(js < 0)])
    n_plus = int(np.sum(js > 0))
    F0 = host(Fsq)[order, :]
    G0 = host(Gsq)
    Fw, Gw = dev(F0), dev(G0)
    Zw = dev(np.eye(P.n))
    rc, done, cnt = ghsvd.block_sweeps(Fw, n_plus, Gw, Zw, 60, block_width=16)
    assert rc == 0 and cnt[done - 1, 2] == 0
    U, V, sf, sg, X = ghsvd.full(Fw, n_plus, Gw, Zw)
    Jsplit = np.where(np.arange(P.n) < n_plus, 1.0, -1.0)
    eF, eG = phase4.decomposition_errors(F0, G0, host(U), host(V), host(sf), host(sg), host(X))
    assert eF < 1e-12 and eG < 1e-12, (eF, eG)
    Uh = host(U)
    UJU = Uh.conj().T @ (Jsplit[:, None] * Uh)
    sgn = np.sign(np.real(np.diag(UJU)))
    assert np.abs(UJU - np.diag(sgn)).max() < 1e-10
    lam = np.sort(sgn * (host(sf) / host(sg)) ** 2)
    st, lam_o, _, _ = oracle.ghsvd(P.F, P.J, P.G, reduce=True, order=1, max_sweeps=80)
    assert st == 0
    assert np.max(np.abs(lam - lam_o) / np.abs(lam_o)) <= 1e-10


def test_full_rank_errors():
    rng = np.random.default_rng(5)
    n = 6
    Fp = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Gp = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Gp[:, 3] = 0.0
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.full(dev(Fp), 3, dev(Gp), dev(np.eye(n)))
    assert e.value.status == -2  # GHSVD_ERANK: a zero column of G'
    Gp[:, 3] = 1.0
    Zs = np.eye(n, dtype=np.complex128)
    Zs[:, 2] = Zs[:, 1]  # singular Z
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.full(dev(Fp), 3, dev(Gp), dev(Zs))
    assert e.value.status == -2  # GHSVD_ERANK: a zero pivot


def test_full_at_full_size():
    # the n = 1024 pencil, in the configuration the benchmark times: the
    # decomposition errors (7.1) and X Z = I on sampled columns (properties
    # that hold at any size; the oracle is not run at this size)
    import bench
    P = synth.workload_pencil(2)
    F = dev(P.F)
    G = dev(P.G)
    J = torch.from_numpy(P.J).cuda()
    r = bench.full_leg(ghsvd, F, J, G, reps=1)
    assert r["sweep_status"] == 0
    assert r["errors_7_1"]["F"] < 1e-12 and r["errors_7_1"]["G"] < 1e-12, r


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 1100, 2100, 4096])
def test_full_inverse_at_many_sizes(n):
    # X = Z^{-1} for Z = Z' Sigma^{-1} at sizes with one tile, a ragged last
    # tile of the blocked solves, and up to the largest n taken; the residual
    # of X Z = I against the backward-stable bound of an LU-based inverse
    rng = np.random.default_rng(100 + n)
    Fp = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Gp = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Zp = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    n_plus = n // 2
    U, V, sf, sg, X = ghsvd.full(dev(Fp), n_plus, dev(Gp), dev(Zp))
    Jd = np.where(np.arange(n) < n_plus, 1.0, -1.0)
    sig = np.sqrt(np.abs(np.sum(np.conj(Fp) * (Jd[:, None] * Fp), axis=0))
                  + np.sum(np.abs(Gp) ** 2, axis=0))
    Z = Zp / sig[None, :]
    Xh = host(X)
    R = Xh @ Z - np.eye(n)
    bound = 8 * n * np.finfo(np.float64).eps * np.linalg.norm(Xh) * np.linalg.norm(Z)
    assert np.linalg.norm(R) <= bound, (np.linalg.norm(R), bound)
    # sigma_f: h_j = f'^* J f' cancels between the rows of either sign of J, so
    # a change of summation order moves it by up to about n eps ||f'_j||^2
    h = np.abs(np.sum(np.conj(Fp) * (Jd[:, None] * Fp), axis=0))
    f2 = np.sum(np.abs(Fp) ** 2, axis=0)
    sfo = np.sqrt(h) / sig
    tol = 4 * n * np.finfo(np.float64).eps * f2 / (np.sqrt(h) * sig) + 1e-15
    assert np.all(np.abs(host(sf) - sfo) <= tol)


def test_full_rejects_n_beyond_largest_order():
    n = 4097
    A = dev(np.eye(n))
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.full(A, 1, A, A)
    assert e.value.status == -1  # GHSVD_EINVAL



def test_full_caller_workspace(oracle):
    # a caller-owned workspace of exactly ghsvd_full_workspace_size(n) bytes
    # gives the same bits as the call that allocates its own; one byte short
    # is GHSVD_ENOMEM; the workspace is reused by a second, smaller call
    P = synth.workload_pencil(4, n_override=97)
    st, Fp, Gp, Zp, _ = oracle.hz_run(P.F, P.J, P.G, max_sweeps=60)
    assert st == 0
    F, G, Z = dev(Fp), dev(Gp), dev(Zp)
    ref = ghsvd.full(F, P.m_plus, G, Z)
    nbytes = ghsvd.full_workspace_size(P.n)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = ghsvd.full(F, P.m_plus, G, Z, work=work)
    for a, b in zip(ref, out):
        assert torch.equal(a, b)
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.full(F, P.m_plus, G, Z, work=work[: nbytes - 256])
    assert e.value.status == -4  # GHSVD_ENOMEM
    Q = synth.workload_pencil(1)
    st, Fq, Gq, Zq, _ = oracle.hz_run(Q.F, Q.J, Q.G, max_sweeps=60)
    ref = ghsvd.full(dev(Fq), Q.m_plus, dev(Gq), dev(Zq))
    out = ghsvd.full(dev(Fq), Q.m_plus, dev(Gq), dev(Zq), work=work)
    for a, b in zip(ref, out):
        assert torch.equal(a, b)
