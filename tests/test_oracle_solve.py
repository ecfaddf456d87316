"""Pins of the oracle's whole sweep method (Algorithm 2 with Section 6.1 inside)
and of its outputs (Section 6.1.7, eq. (3.2)).

Each pin is independent of the oracle's code: library routines on special
cases, 40-digit brute force on tiny pencils, invariants evaluated on the
factors, equivariances of the generalized eigenproblem, and the sweep counts
the paper reports as plausible.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1907_08560_amd import synth

EPS = 2.0 ** -52


def brute_force(F, J, G, dps=40):
    """Eigenvalues of (F^* J F, G^* G) in `dps`-digit arithmetic: H and S formed
    from the double inputs, S = L L^*, eig of L^-1 H L^-*, ascending."""
    mp.mp.dps = dps
    m, n = F.shape
    p = G.shape[0]
    Fm = mp.matrix(m, n)
    Gm = mp.matrix(p, n)
    for i in range(m):
        for j in range(n):
            Fm[i, j] = mp.mpc(F[i, j].real, F[i, j].imag) * int(J[i])
    Fr = mp.matrix(m, n)
    for i in range(m):
        for j in range(n):
            Fr[i, j] = mp.mpc(F[i, j].real, F[i, j].imag)
    for i in range(p):
        for j in range(n):
            Gm[i, j] = mp.mpc(G[i, j].real, G[i, j].imag)
    H = Fr.transpose_conj() * Fm
    S = Gm.transpose_conj() * Gm
    L = mp.cholesky(S)
    Li = mp.inverse(L)
    C = Li * H * Li.transpose_conj()
    C = (C + C.transpose_conj()) / 2
    E = mp.eighe(C, eigvals_only=True)
    return np.array(sorted(float(mp.re(e)) for e in E))


def rel_err(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


def small_pencil(seed, n, s_lo, ratio_m=1.5, ratio_p=2.0, plus=0.75, j_identity=False):
    m = int(math.ceil(ratio_m * n))
    p = int(math.ceil(ratio_p * n))
    return synth.random_pencil(seed, n, m, int(round(plus * m)), p, s_lo, j_identity=j_identity)


# --- P2: special cases that reduce to a library routine ------------------------------

def test_G_identity_J_identity_is_svd(oracle):
    rng = np.random.default_rng(1)
    F = rng.standard_normal((30, 20)) + 1j * rng.standard_normal((30, 20))
    st, lam, X, stats = oracle.ghsvd(F, np.ones(30), np.eye(20, dtype=complex))
    assert st == 0
    sv = np.linalg.svd(F, compute_uv=False)
    assert rel_err(lam, np.sort(sv ** 2)) < 1e-13


def test_G_identity_is_hermitian_eig(oracle):
    rng = np.random.default_rng(2)
    F = rng.standard_normal((30, 20)) + 1j * rng.standard_normal((30, 20))
    J = np.where(np.arange(30) < 18, 1, -1)
    st, lam, X, stats = oracle.ghsvd(F, J, np.eye(20, dtype=complex))
    assert st == 0
    ref = np.linalg.eigvalsh(F.conj().T @ (J[:, None] * F))
    assert np.max(np.abs(lam - ref)) < 1e-12 * np.max(np.abs(ref))


def test_J_identity_is_generalized_eig(oracle):
    P = small_pencil(3, 24, 1e-1, j_identity=True)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G)
    assert st == 0 and np.all(lam > 0)
    ref = sl.eigh(P.F.conj().T @ P.F, P.G.conj().T @ P.G, eigvals_only=True)
    assert rel_err(lam, ref) < 1e-12


def test_F_equals_G_gives_ones(oracle):
    P = small_pencil(4, 20, 1e-3)
    # A fully degenerate spectrum: any rotation inside it is an exact solution, so
    # the 2x2 steps may keep rotating at rounding level and never count as "small";
    # the stop rule may then end on the sweep cap (status 1), outputs still valid.
    st, lam, X, stats = oracle.ghsvd(P.G, np.ones(P.p), P.G)
    assert st in (0, 1)
    assert np.max(np.abs(lam - 1.0)) < 1e-12


def test_order_one(oracle):
    f = np.array([[1.0 + 2j], [3.0 - 1j], [0.5j]])
    g = np.array([[2.0 + 0j], [1j]])
    J = np.array([1, -1, 1])
    st, lam, X, _ = oracle.ghsvd(f, J, g)
    a = 5.0 - 10.0 + 0.25
    assert st == 0 and abs(lam[0] - a / 5.0) < 1e-15
    assert abs(abs(X[0, 0]) - 1 / math.sqrt(5.0)) < 1e-15


def test_order_two_closed_form(oracle):
    rng = np.random.default_rng(7)
    for _ in range(10):
        F = rng.standard_normal((4, 2)) + 1j * rng.standard_normal((4, 2))
        G = rng.standard_normal((3, 2)) + 1j * rng.standard_normal((3, 2))
        J = np.array([1, -1, 1, -1])
        H = F.conj().T @ (J[:, None] * F)
        S = G.conj().T @ G
        A2 = (S[0, 0] * S[1, 1] - abs(S[0, 1]) ** 2).real
        A1 = -(H[0, 0] * S[1, 1] + H[1, 1] * S[0, 0] - 2 * (H[0, 1] * np.conj(S[0, 1])).real).real
        A0 = (H[0, 0] * H[1, 1] - abs(H[0, 1]) ** 2).real
        r = np.sort(np.roots([A2, A1, A0]).real)
        st, lam, X, _ = oracle.ghsvd(F, J, G)
        assert st == 0 and rel_err(lam, r) < 1e-13


# --- P3: high-precision brute force ------------------------------------------------

@pytest.mark.parametrize("seed,n,s_lo,bound", [(21, 16, 1e-4, 1e-12), (22, 24, 1e-6, 1e-10),
                                                (23, 20, 1e-2, 1e-12)])
def test_brute_force(oracle, seed, n, s_lo, bound):
    P = small_pencil(seed, n, s_lo)
    ref = brute_force(P.F, P.J, P.G)
    for reduce, order in ((False, 0), (False, 1), (True, 1)):
        st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G, reduce=reduce, order=order)
        assert st == 0
        assert rel_err(lam, ref) < bound, (reduce, order, rel_err(lam, ref))


def test_brute_force_ill_conditioned_band(oracle):
    # cond(S) = 1e16: the error bound degrades with kappa(G) (about eps * kappa(G)).
    P = small_pencil(24, 20, 1e-8)
    ref = brute_force(P.F, P.J, P.G)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G)
    assert st == 0
    assert rel_err(lam, ref) < 1e-7


# --- P4: invariants on the factors -------------------------------------------------

def invariants(F, J, G, lam, X):
    n = X.shape[1]
    GX = G @ X
    FX = F @ X
    e_s = np.abs(GX.conj().T @ GX - np.eye(n)).max()
    Hx = FX.conj().T @ (J[:, None] * FX)
    off = Hx - np.diag(np.diag(Hx))
    scale = np.sqrt(np.outer(np.abs(lam), np.abs(lam))) + 1e-300
    e_h = np.max(np.abs(off) / np.maximum(scale, np.abs(lam).max() * 1e-16))
    e_d = np.max(np.abs(np.real(np.diag(Hx)) - lam) / np.abs(lam))
    # residual F^*(J F X) - G^*(G X) diag(lam), relative
    R = F.conj().T @ (J[:, None] * FX) - G.conj().T @ (GX * lam[None, :])
    e_r = np.linalg.norm(R) / (np.linalg.norm(F) ** 2 * np.linalg.norm(X) ** 2
                               + np.linalg.norm(G) ** 2 * np.linalg.norm(X) ** 2 * np.abs(lam).max())
    return e_s, e_h, e_d, e_r


@pytest.mark.parametrize("reduce", [False, True])
def test_invariants_workload_one(oracle, reduce):
    P = synth.workload_pencil(1)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G, reduce=reduce, order=1)
    assert st == 0
    e_s, e_h, e_d, e_r = invariants(P.F, P.J, P.G, lam, X)
    assert e_s < 1e-11 and e_h < 1e-11 and e_d < 1e-11 and e_r < 1e-14, (e_s, e_h, e_d, e_r)


def test_inertia_matches_H(oracle):
    # The number of negative eigenvalues equals the inertia of H = F^* J F (Sylvester),
    # which differs from the count of -1 entries of J for a tall F.
    P = synth.workload_pencil(1)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G)
    H = P.F.conj().T @ (P.J[:, None] * P.F)
    nu = int((np.linalg.eigvalsh(H) < 0).sum())
    assert int((lam < 0).sum()) == nu
    assert nu != int((P.J < 0).sum())


# --- P5: equivariances ---------------------------------------------------------------

def test_equivariances(oracle):
    P = small_pencil(31, 24, 1e-4)
    st, lam, X, _ = oracle.ghsvd(P.F, P.J, P.G)
    rng = np.random.default_rng(9)
    # column permutation
    pm = rng.permutation(P.n)
    _, lam2, X2, _ = oracle.ghsvd(P.F[:, pm], P.J, P.G[:, pm])
    assert rel_err(lam2, lam) < 1e-12
    # (alpha F, beta G) -> (alpha / beta)^2 lambda
    _, lam3, _, _ = oracle.ghsvd(3.0 * P.F, P.J, 0.25 * P.G)
    assert rel_err(lam3, lam * 144.0) < 1e-12
    # column scaling F D, G D
    d = 10.0 ** rng.uniform(-3, 3, P.n)
    _, lam4, _, _ = oracle.ghsvd(P.F * d, P.J, P.G * d)
    assert rel_err(lam4, lam) < 1e-12
    # unitary Q on G's rows
    Q = synth.haar_frame(rng, P.p, P.p)
    _, lam5, _, _ = oracle.ghsvd(P.F, P.J, Q @ P.G)
    assert rel_err(lam5, lam) < 1e-12
    # unitary within each sign block of F (keeps F^* J F)
    mp_ = P.m_plus
    Qp = synth.haar_frame(rng, mp_, mp_)
    Qm = synth.haar_frame(rng, P.m - mp_, P.m - mp_)
    F6 = np.vstack([Qp @ P.F[:mp_], Qm @ P.F[mp_:]])
    _, lam6, _, _ = oracle.ghsvd(F6, P.J, P.G)
    assert rel_err(lam6, lam) < 1e-12
    # row order of F with J permuted alike
    rp = rng.permutation(P.m)
    _, lam7, _, _ = oracle.ghsvd(P.F[rp], P.J[rp], P.G)
    assert rel_err(lam7, lam) < 1e-12


def test_orderings_agree(oracle):
    P = small_pencil(32, 30, 1e-5)
    _, lam0, _, s0 = oracle.ghsvd(P.F, P.J, P.G, order=0)
    _, lam1, _, s1 = oracle.ghsvd(P.F, P.J, P.G, order=1)
    assert rel_err(lam1, lam0) < 1e-11


# --- P6: plausibility of the sweep counts --------------------------------------------

def test_sweep_counts_plausible(oracle):
    P = synth.workload_pencil(1)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G, order=1)
    assert st == 0 and 8 <= stats[0] <= 30
    assert stats[4] == 0  # the final sweep applied no big transformation
    assert stats[1] == stats[0] * P.n * (P.n - 1) // 2


# --- status paths --------------------------------------------------------------------

def test_not_converged_status(oracle):
    P = synth.workload_pencil(1)
    st, lam, X, stats = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=1)
    assert st == 1 and stats[0] == 1


def test_rank_deficient_G(oracle):
    P = small_pencil(33, 10, 1e-2)
    G = P.G.copy()
    G[:, 3] = G[:, 7]
    st, *_ = oracle.ghsvd(P.F, P.J, G)
    assert st == -2
    G[:, 3] = 0
    st, *_ = oracle.ghsvd(P.F, P.J, G)
    assert st == -2


def test_nonfinite_input(oracle):
    P = small_pencil(34, 10, 1e-2)
    F = P.F.copy()
    F[2, 2] = np.nan
    st, *_ = oracle.ghsvd(F, P.J, P.G)
    assert st == -3


def test_literal_criterion_same_result(oracle):
    P = small_pencil(35, 24, 1e-4)
    _, lam0, _, _ = oracle.ghsvd(P.F, P.J, P.G, crit_literal=0)
    _, lam1, _, _ = oracle.ghsvd(P.F, P.J, P.G, crit_literal=1)
    assert rel_err(lam1, lam0) < 1e-11
