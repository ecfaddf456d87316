"""Pins of the oracle's Level-2 blocked sweeps (Section 6.4): BO (one inner
sweep per block pivot) under both inner orderings, and FB (inner sweeps until
one applies no big transformation, at most 30).

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
