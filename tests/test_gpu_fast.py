"""GPU parity of the explicit-formation route (Section 4.5: H = F^* J F and
S = G^* G formed, S = R^* R, C = R^{-*} H R^{-1}, Jacobi on C, X = R^{-1} V)
against the oracle's formation with the library eigensolver.

Tolerance: forming S and reducing to C perturbs C by about eps cond(S) ||C||
(each side), so by Weyl's bound every eigenvalue moves by at most that much;
the gate is n eps cond(S) max|lambda| for the difference of the two sides.  X
is checked through the pencil (X^* S X = I, X^* H X = diag(lambda), each within
the same relative bound) and, for eigenvalues whose relative gap exceeds 1e-3,
column by column against the oracle's up to a phase.  Pencils with cond(S)
above the caller's bound take the implicit HZ path, whose result must be
bitwise that of ghsvd_solve with the same options.
"""
import numpy as np
import pytest
import torch

from oracle import fast as FX
from paper_1907_08560_amd import ghsvd, synth
from gpu_util import host, to_dev

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


def check(P, lam, X, tag):
    lo, Xo, R, C = FX.solve_explicit(P.F, P.J, P.G)
    H = P.F.conj().T @ (P.J.astype(float)[:, None] * P.F)
    S = P.G.conj().T @ P.G
    kap = np.linalg.cond(S)
    n = P.n
    lam, X = host(lam), host(X)
    scale = np.abs(lo).max()
    gate = n * EPS * kap * scale
    err = np.abs(lam - lo).max()
    assert err <= gate, (tag, err, gate)
    tol = n * EPS * kap
    assert np.abs(X.conj().T @ S @ X - np.eye(n)).max() <= tol, tag
    XH = X.conj().T @ H @ X
    assert np.abs(XH - np.diag(lam)).max() <= tol * scale, tag
    gaps = np.full(n, np.inf)
    if n > 1:
        d = np.diff(lo)
        gaps[:-1] = np.minimum(gaps[:-1], d)
        gaps[1:] = np.minimum(gaps[1:], d)
    for j in np.nonzero(gaps > 1e-3 * scale)[0]:
        ph = np.vdot(X[:, j], Xo[:, j])
        ph = ph / abs(ph) if abs(ph) > 0 else 1.0
        assert np.abs(X[:, j] * ph - Xo[:, j]).max() <= 1e-8 * np.abs(Xo[:, j]).max(), (tag, j)
    print(f"{tag}: n={n} cond(S)={kap:.1e} max |dlambda| = {err:.2e} (gate {gate:.1e})",
          flush=True)


@pytest.mark.parametrize("seed,n,s_lo", [(1, 1, 0.5), (2, 2, 0.5), (3, 17, 0.3), (4, 64, 0.2),
                                         (5, 65, 0.2), (6, 130, 0.1), (7, 257, 0.1),
                                         (8, 513, 0.05)])
def test_fast_route_matches_oracle(seed, n, s_lo):
    P = synth.random_pencil(seed, n, int(np.ceil(1.5 * n)), int(np.ceil(1.1 * n)), 2 * n, s_lo)
    F, J, G = to_dev(P)
    lam, X, info = ghsvd.solve_fast(F, J, G, cond_max=1e6)
    assert info["status"] == 0 and info["path"] == "fast", info
    check(P, lam, X, f"seed {seed}")


def test_fast_route_square_and_definite():
    # square factors (the reduced shape) and J = I (a definite H)
    P = synth.random_pencil(11, 200, 200, 150, 200, 0.1)
    F, J, G = to_dev(P)
    lam, X, info = ghsvd.solve_fast(F, J, G, cond_max=1e6)
    assert info["path"] == "fast" and info["status"] == 0
    check(P, lam, X, "square")
    P = synth.random_pencil(12, 150, 225, 225, 300, 0.1, j_identity=True)
    F, J, G = to_dev(P)
    lam, X, info = ghsvd.solve_fast(F, J, G, cond_max=1e6)
    assert info["path"] == "fast" and np.all(host(lam) > 0)
    check(P, lam, X, "J = I")


def test_ill_conditioned_pencil_falls_back_to_hz():
    P = synth.workload_pencil(4, 3, n_override=300)  # cond(S) up to 1e12
    F, J, G = to_dev(P)
    kw = dict(precision="fp64", variant="blocked")
    lam, X, info = ghsvd.solve_fast(F, J, G, cond_max=1e4, fallback=kw)
    assert info["path"] == "hz" and info["status"] == 0 and info["cond_est"] > 1e4
    lam2, X2, info2 = ghsvd.solve(F, J, G, **kw)
    assert torch.equal(lam, lam2) and torch.equal(X, X2)
    assert info["hz"]["sweeps_fp64"] == info2["sweeps_fp64"]
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.solve_fast(F, J, G, cond_max=1e4)
    assert e.value.status == -2


def test_singular_s_is_rejected():
    P = synth.random_pencil(13, 40, 60, 45, 80, 0.2)
    P.G[:, 7] = 0.0  # S singular: the factorization meets a zero pivot
    F, J, G = to_dev(P)
    with pytest.raises(ghsvd.GhsvdError) as e:
        ghsvd.solve_fast(F, J, G, cond_max=1e30)
    assert e.value.status == -2


def test_phase1_output_through_fast_route():
    T, H, U = synth.phase1_set(61, 3, "B", 12, 50)
    F, J, G, stats = ghsvd.phase1(ghsvd.atoms_to_device(T), ghsvd.to_device_fortran(H),
                                  torch.from_numpy(np.ascontiguousarray(U.T)).cuda())
    lam, X, info = ghsvd.solve_fast(F, J, G, cond_max=1e8)
    assert info["path"] == "fast" and info["status"] == 0

    class P:  # the assembled pencil on the host
        pass
    P.F, P.J, P.G, P.n = host(F), host(J), host(G), 50
    check(P, lam, X, "phase 1 -> fast")
