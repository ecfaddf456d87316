"""Pins of the oracle's full GHSVD (Phase 4, Section 7; the outputs of
Section 6.1) against properties the mathematics fixes."""
import itertools

import numpy as np

from oracle import phase4
from paper_1907_08560_amd import synth


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_lu_complete_reconstructs_and_pivots_brute_force():
    rng = np.random.default_rng(11)
    A = crandn(rng, 7, 7)
    LU, rows, cols = phase4.lu_complete(A)
    L = np.tril(LU, -1) + np.eye(7)
    U = np.triu(LU)
    assert np.abs(A[np.ix_(rows, cols)] - L @ U).max() < 1e-14 * np.abs(A).max() * 7
    # complete pivoting: |l_ij| <= 1, and every pivot is the largest entry of
    # its Schur complement (recomputed by brute force from A)
    assert np.abs(np.tril(LU, -1)).max() <= 1.0 + 1e-15
    for k in range(7):
        S = A[np.ix_(rows, cols)][k:, k:] - L[k:, :k] @ U[:k, k:]
        assert np.isclose(abs(U[k, k]), np.abs(S).max(), rtol=1e-13)


def test_lu_complete_tie_rule():
    # equal moduli everywhere: the first entry in column-major order wins,
    # so no interchange happens at the first step
    A = np.array([[1, -1j], [1j, 1]], dtype=np.complex128) + 0.0
    A[1, 1] = 2.0  # make the matrix nonsingular; the second step is forced
    LU, rows, cols = phase4.lu_complete(A)
    assert rows[0] == 1 and cols[0] == 1  # the unique maximum 2 at (1, 1)
    B = np.array([[1, 1], [1, -1]], dtype=np.complex128)
    LU, rows, cols = phase4.lu_complete(B)
    assert rows[0] == 0 and cols[0] == 0


def test_inverse_from_lu():
    rng = np.random.default_rng(12)
    for n in (1, 2, 5, 30):
        A = crandn(rng, n, n)
        X = phase4.inverse_from_lu(*phase4.lu_complete(A))
        assert np.abs(X @ A - np.eye(n)).max() < 1e-12 * np.linalg.cond(A)


def test_textbook_special_cases():
    # F = G, J = I: every generalized singular value pair is (1/sqrt 2, 1/sqrt 2),
    # U = V, and the decomposition reproduces F exactly in exact arithmetic
    rng = np.random.default_rng(13)
    Q, _ = np.linalg.qr(crandn(rng, 6, 6))
    Fp = Q * np.array([2.0, 1.0, 3.0, 0.5, 1.5, 4.0])[None, :]
    U, V, sf, sg, X = phase4.full_ghsvd(Fp, np.ones(6), Fp, np.eye(6))
    assert np.allclose(sf, 1 / np.sqrt(2)) and np.allclose(sg, 1 / np.sqrt(2))
    assert np.abs(U - V).max() == 0.0
    eF, eG = phase4.decomposition_errors(Fp, Fp, U, V, sf, sg, X)
    assert eF < 1e-15 and eG < 1e-15
    # diagonal pencil: Z' = I, F' = diag(a) (J = diag(s)), G' = diag(b):
    # sigma_f / sigma_g = |a| / |b|, X = diag(sqrt(a^2 + b^2))
    a = np.array([3.0, -1.0, 0.5]) + 0j
    b = np.array([4.0, 2.0, 1.0]) + 0j
    U, V, sf, sg, X = phase4.full_ghsvd(np.diag(a), np.array([1, -1, 1]), np.diag(b), np.eye(3))
    assert np.allclose(sf / sg, np.abs(a) / np.abs(b), rtol=1e-15)
    assert np.allclose(X, np.diag(np.sqrt(np.abs(a) ** 2 + np.abs(b) ** 2)), rtol=1e-15)


def test_full_ghsvd_on_converged_sweeps(oracle):
    # the oracle's own converged sweeps on workload 1's tall factors: the
    # paper's structure of the outputs and the relative errors (7.1)
    P = synth.workload_pencil(1)
    st, Fp, Gp, Zp, stats = oracle.hz_run(P.F, P.J, P.G, max_sweeps=40)
    assert st == 0
    U, V, sf, sg, X = phase4.full_ghsvd(Fp, P.J, Gp, Zp)
    n = P.n
    assert np.abs(sf ** 2 + sg ** 2 - 1.0).max() < 1e-15
    UJU = U.conj().T @ (P.J[:, None] * U)
    assert np.abs(UJU - np.diag(np.sign(np.real(np.diag(UJU))))).max() < 1e-12
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
    eF, eG = phase4.decomposition_errors(P.F, P.G, U, V, sf, sg, X)
    assert eF < 1e-13 and eG < 1e-13, (eF, eG)
    # the generalized eigenvalues of (F^* J F, G^* G) are +-(sigma_f / sigma_g)^2
    lam = np.sort(np.sign(np.real(np.diag(UJU))) * (sf / sg) ** 2)
    st2, lam_o, _, _ = oracle.ghsvd(P.F, P.J, P.G, max_sweeps=40)
    assert st2 == 0
    assert np.abs(lam - lam_o).max() <= 1e-12 * np.abs(lam_o).max()


def test_permutation_bookkeeping_against_brute_force():
    # every small permutation pair: the inverse is unique, whatever the pivots
    rng = np.random.default_rng(14)
    A = crandn(rng, 3, 3)
    X = phase4.inverse_from_lu(*phase4.lu_complete(A))
    for pr, pc in itertools.product(itertools.permutations(range(3)), repeat=2):
        B = A[np.ix_(pr, pc)]
        XB = phase4.inverse_from_lu(*phase4.lu_complete(B))
        # B = P A Q  =>  B^{-1} = Q^T A^{-1} P^T
        assert np.abs(XB - X[np.ix_(pc, pr)]).max() < 1e-13 * np.abs(X).max()
