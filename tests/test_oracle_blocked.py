"""Pins of the oracle's Level-2 blocked sweeps (Section 6.4): BO (one inner
sweep per block pivot) under both inner orderings, and FB (inner sweeps until
one applies no transformation at all, big or small, at most 30: Section
6.1.7 on the inner levels of a blocked algorithm).

Cross ordering: with full blocks, the first block step of a sweep visits all
pairs inside every block and the other steps only the w x w pairs across the
two blocks, so a block sweep visits each of the n(n-1)/2 column pairs exactly
once; the full ordering revisits the pairs inside a block at every block step.
Both converge to the eigenvalues of the pointwise iteration.
"""
import numpy as np
import pytest

from paper_1907_08560_amd import synth


def _pencil(seed, n, s_lo):
    m, p = int(1.5 * n), 2 * n
    return synth.random_pencil(seed, n, m, int(round(0.75 * m)), p, s_lo)


def test_cross_visits_each_pair_once_per_sweep(oracle):
    n, w = 64, 8
    P = _pencil(911, n, 1e-2)
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=1, inner_order=1)
    assert st in (0, 1)
    assert stats[1] == n * (n - 1) // 2
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=1, inner_order=0)
    nb = n // w
    assert stats[1] == (nb - 1) * (nb // 2) * (2 * w) * (2 * w - 1) // 2


@pytest.mark.parametrize("inner", [0, 1, 2])
def test_blocked_orderings_reach_pointwise_eigenvalues(oracle, inner):
    n, w = 48, 8
    P = _pencil(913, n, 1e-3)
    st, lam_ref, _, _ = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=60)
    assert st == 0
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=60, inner_order=inner)
    assert st == 0
    st, lam, X = oracle.hz_post(F, P.J, G, Z)
    assert st == 0
    assert np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)) < 1e-11


def test_fb_on_one_block_pair_is_a_full_solve(oracle):
    # n = 2w: the only block pivot is the whole pencil, so FB's inner sweeps
    # are the pointwise iteration itself.  The first block sweep runs them to
    # convergence (a whole number of inner sweeps over the c(c-1)/2 pairs,
    # more than one), the second applies no big transformation and stops the
    # iteration, and the swept factors are J-orthogonal / orthogonal to the
    # tolerance of (6.12).  BO on the same pencil needs many block sweeps.
    n, w = 16, 8
    P = _pencil(917, n, 1e-2)
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=1, inner_order=2)
    pairs = n * (n - 1) // 2
    assert stats[1] % pairs == 0 and stats[1] > pairs
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=60, inner_order=2)
    assert st == 0 and stats[0] == 2
    H = F.conj().T @ (P.J[:, None] * F)
    S = G.conj().T @ G
    dh = np.sqrt(np.abs(np.diag(H)))
    ds = np.sqrt(np.abs(np.diag(S)))
    off = lambda M, d: np.max(np.abs(M - np.diag(np.diag(M))) / np.outer(d, d))
    assert off(H, dh) < 1e-13 and off(S, ds) < 1e-13
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=60, inner_order=0)
    assert st == 0 and stats[0] > 2


def shortened_pivot(o, F, J, G):
    """The (J)QR-shortened block pivot (Section 6.4.2) of the columns of (F, G),
    with the columns put back in pivot order: (F~, J^, G~), F~^* J^ F~ = F^* J F,
    G~^* G~ = G^* G."""
    st, A, Jh, perm, _, _ = o.jqr(F, J)
    assert st == 0
    st, R = o.qr(np.asfortranarray(G[:, perm]))
    assert st == 0
    c = F.shape[1]
    Ft = np.zeros((c, c), dtype=np.complex128)
    Gt = np.zeros((c, c), dtype=np.complex128)
    Ft[:, perm] = A
    Gt[:, perm] = R
    return np.asfortranarray(Ft), Jh, np.asfortranarray(Gt)


@pytest.mark.parametrize("seed,n,s_lo", [(917, 16, 1e-2), (919, 24, 1e-4), (921, 32, 1e-3)])
def test_fb_inner_level_is_algorithm_2(oracle, seed, n, s_lo):
    # n = 2w: the only block pivot is the whole pencil, so the FB inner level
    # of the first block sweep is Algorithm 2 itself, run on the shortened
    # pivot with the round-robin ordering and Algorithm 2's own stopping test
    # (a sweep with no transformation, big or small).  The visited pairs, the
    # number of inner sweeps and the accumulated Z^ must be those of the
    # pointwise iteration with that test; the "no big transformation" test
    # of the outer level stops earlier on these pencils.
    w = n // 2
    P = _pencil(seed, n, s_lo)
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=1, inner_order=2)
    assert st in (0, 1)
    Ft, Jh, Gt = shortened_pivot(oracle, P.F, P.J, P.G)
    st1, _, _, Zp, s1 = oracle.hz_run(Ft, Jh, Gt, order=1, max_sweeps=30, stop_rule=1)
    st0, _, _, _, s0 = oracle.hz_run(Ft, Jh, Gt, order=1, max_sweeps=30, stop_rule=0)
    assert st1 == 0 and s1[4] == 0
    pairs = n * (n - 1) // 2
    assert stats[1] == s1[1] == s1[0] * pairs
    assert stats[5] == s1[0]
    assert stats[2] == s1[2] and stats[3] == s1[3]
    assert s0[0] < s1[0]  # the two stopping tests differ on this pencil
    # F = F_in Z^, G = G_in Z^, Z = Z^ with Z^ the pointwise run's accumulation
    for A, B in ((F, P.F @ Zp), (G, P.G @ Zp), (Z, Zp)):
        err = np.max(np.abs(A - B)) / np.max(np.abs(B))
        assert err < 1e-12, err



@pytest.mark.parametrize("inner", [3, 4])
def test_three_level_runs_reach_pointwise_eigenvalues(oracle, inner):
    n, w = 48, 16
    P = _pencil(923, n, 1e-3)
    st, lam_ref, _, _ = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=60)
    assert st == 0
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=60, inner_order=inner)
    assert st == 0
    st, lam, X = oracle.hz_post(F, P.J, G, Z)
    assert st == 0
    assert np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)) < 1e-11


def test_three_level_bo_visits_one_nested_sweep(oracle):
    # n = 2w = 32: one block pivot, shortened to 32 x 32 and swept once by a
    # Level-2 run of width 8: 4 blocks, 3 block steps of 2 block pivots of 16
    # columns, each visited once in the full round-robin order (120 pairs)
    P = _pencil(925, 32, 1e-2)
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=16, max_sweeps=1, inner_order=3)
    assert st in (0, 1)
    assert stats[1] == 3 * 2 * (16 * 15 // 2) and stats[5] == 1


@pytest.mark.parametrize("seed,n,s_lo", [(927, 32, 1e-2), (929, 32, 1e-4)])
def test_three_level_fb_inner_level_is_a_converged_level2_run(oracle, seed, n, s_lo):
    # n = 2w: the inner level of the first block sweep is the Level-2 blocked
    # run (width 8, BO inner) on the shortened pivot, run until a blocked
    # sweep applies no big transformation; a single nested sweep (BO) differs
    w = n // 2
    P = _pencil(seed, n, s_lo)
    st, F, G, Z, stats = oracle.hz_block_run(P.F, P.J, P.G, w=w, max_sweeps=1, inner_order=4)
    assert st in (0, 1)
    Ft, Jh, Gt = shortened_pivot(oracle, P.F, P.J, P.G)
    st1, _, _, Zp, s1 = oracle.hz_block_run(Ft, Jh, Gt, w=8, max_sweeps=30, inner_order=0)
    assert st1 == 0 and s1[0] > 1
    assert stats[1] == s1[1] and stats[5] == s1[0]
    assert stats[2] == s1[2] and stats[3] == s1[3]
    for A, B in ((F, P.F @ Zp), (G, P.G @ Zp), (Z, Zp)):
        err = np.max(np.abs(A - B)) / np.max(np.abs(B))
        assert err < 1e-12, err
