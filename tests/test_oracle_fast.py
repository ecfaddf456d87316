"""Pins of the explicit-formation oracle (Section 4.5).

Checked against what the mathematics fixes:
  * a pencil of diagonal F and G has lambda_j = J_j f_j^2 / g_j^2 and X
    diagonal with X^* S X = I (closed form);
  * on well-conditioned random pencils the eigenvalues agree with the
    implicit HZ oracle (one-sided Jacobi on the factors, never forming H or
    S) to eps cond(S) and satisfy H X = S X diag(lambda), X^* S X = I;
  * the Cholesky factor is upper triangular with a positive diagonal and
    R^* R = S;
  * each planted mistake (MUTANT 1..4) fails one of these.
"""
import numpy as np
import pytest

from oracle import fast as FX
from oracle import oracle as O
from paper_1907_08560_amd import synth


def diag_pencil():
    f = np.array([2.0, -1.0, 0.5, 3.0])
    g = np.array([1.0, 2.0, 0.25, 1.5])
    J = np.array([1, -1, 1, -1], dtype=np.int8)
    F = np.vstack([np.diag(f).astype(complex), np.zeros((2, 4))])
    J6 = np.concatenate([J, np.array([1, -1], dtype=np.int8)])
    G = np.diag(g).astype(complex)
    return F, J6, G, J * f * f / (g * g)


def pencil_ok(F, J, G, lam, X, tol):
    H, S = F.conj().T @ (J.astype(float)[:, None] * F), G.conj().T @ G
    n = X.shape[1]
    res = np.abs(H @ X - S @ X * lam[None, :]).max() / (np.abs(H).max() * np.abs(X).max())
    orth = np.abs(X.conj().T @ S @ X - np.eye(n)).max()
    return res < tol and orth < tol and np.all(np.diff(lam) >= 0)


def test_closed_form_diagonal_pencil():
    F, J, G, ref = diag_pencil()
    lam, X, R, C = FX.solve_explicit(F, J, G)
    np.testing.assert_allclose(lam, np.sort(ref), rtol=1e-14)
    assert np.all((np.abs(X) > 0).sum(axis=0) == 1)  # one nonzero per column
    assert pencil_ok(F, J, G, lam, X, 1e-14)


@pytest.mark.parametrize("seed,n,s_lo", [(1, 12, 0.3), (2, 40, 0.1), (3, 65, 0.05)])
def test_matches_implicit_hz(seed, n, s_lo):
    P = synth.random_pencil(seed, n, int(1.5 * n), int(1.1 * n), 2 * n, s_lo)
    lam, X, R, C = FX.solve_explicit(P.F, P.J, P.G)
    S = P.G.conj().T @ P.G
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.real(np.diag(R)) > 0)
    assert np.abs(R.conj().T @ R - S).max() <= 1e-13 * np.abs(S).max()
    st, lh, Xh, stats = O.Oracle().ghsvd(P.F, P.J, P.G, reduce=True, order=0, max_sweeps=60)
    assert st == 0
    kap = np.linalg.cond(S)
    np.testing.assert_allclose(lam, np.sort(lh), rtol=1e-13 * kap * n, atol=0)
    assert pencil_ok(P.F, P.J, P.G, lam, X, 1e-12 * kap)


def battery():
    fails = []
    F, J, G, ref = diag_pencil()
    lam, X, _, _ = FX.solve_explicit(F, J, G)
    if not np.allclose(lam, np.sort(ref), rtol=1e-14) or not pencil_ok(F, J, G, lam, X, 1e-13):
        fails.append("diag")
    P = synth.random_pencil(4, 16, 24, 18, 32, 0.2)
    lam, X, _, _ = FX.solve_explicit(P.F, P.J, P.G)
    if not pencil_ok(P.F, P.J, P.G, lam, X, 1e-11):
        fails.append("random")
    return fails


@pytest.mark.parametrize("mutant", range(1, 5))
def test_planted_mistakes_are_caught(mutant, monkeypatch):
    assert battery() == []
    monkeypatch.setattr(FX, "MUTANT", mutant)
    assert battery() != [], f"mutant {mutant} not caught"
