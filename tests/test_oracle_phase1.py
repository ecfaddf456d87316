"""Pins of the Phase 1 oracle (Section 4: ZHEBPJ and the assembly of F~, J~, G~).

The oracle is checked against what the mathematics fixes, not against itself:
  * the factorization reproduces T (T = Mt^* Jt Mt) and, by Sylvester's law of
    inertia, Jt has as many +1 and -1 as T has positive and negative
    eigenvalues (numpy's eigvalsh);
  * the signs come positive first (Section 4.3);
  * every pivot obeys the Bunch-Parlett rule on the Schur complement, which
    the test recomputes from T alone with numpy's solver (an independent
    route to the same matrix);
  * closed forms: a diagonal T, the 2x2 [[0, 2], [2, 0]], a singular T;
  * the assembly satisfies eq. (4.2): F~^* J~ F~ = sum_a H_a^* T_a H_a and
    G~^* G~ = sum_a S_a^* S_a;
  * end to end, the GHSVD of (F~, J~, G~) by the HZ oracle gives the
    eigenvalues of the pencil (H, S) that scipy's generalized eigensolver
    finds;
  * each planted mistake (MUTANT 1..6) fails at least one of these.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from oracle import phase1 as P1
from paper_1907_08560_amd import synth

ALPHA = (1.0 + math.sqrt(17.0)) / 8.0


def atom(kind, nl, a=0, n=8, seed=7, atoms=4):
    return synth.phase1_atom(seed, atoms, a, kind, nl, n)


def check_pivots(T, perm, blocks):
    """Every pivot against the Bunch-Parlett rule on the Schur complement
    recomputed from T: S = T[R, R] - T[R, E] T[E, E]^{-1} T[E, R] with E the
    indices eliminated so far and R the rest (in pivoted order)."""
    r = T.shape[0]
    for k, s in blocks:
        E = list(perm[:k])
        R = list(perm[k:])
        S = T[np.ix_(R, R)]
        if E:
            S = S - T[np.ix_(R, E)] @ np.linalg.solve(T[np.ix_(E, E)], T[np.ix_(E, R)])
        d = np.abs(np.real(np.diagonal(S)))
        off = np.abs(S - np.diag(np.diagonal(S)))
        mu0 = max(d.max(), off.max())
        if s == 0:
            assert mu0 < 1e-12 * np.abs(T).max()
            return
        rel = 1e-9 * mu0
        if s == 1:
            assert d.max() >= ALPHA * mu0 - rel, (k, d.max(), mu0)
            assert d[0] >= d.max() - rel  # the chosen one sits at position k
        else:
            assert d.max() < ALPHA * mu0 + rel, (k, d.max(), mu0)
            assert off[0, 1] >= off.max() - rel
    assert sum(s for _, s in blocks) == r


def factor_ok(T, Mt, Jt, tol=1e-12):
    rec = Mt.conj().T @ (Jt.astype(float)[:, None] * Mt)
    ev = np.linalg.eigvalsh(T)
    sc = np.abs(ev).max() * 1e-10
    return (np.abs(rec - T).max() <= tol * max(np.abs(T).max(), 1e-300) and
            int((Jt > 0).sum()) == int((ev > sc).sum()) and
            int((Jt < 0).sum()) == int((ev < -sc).sum()) and
            np.all(np.diff(np.where(Jt > 0, 0, np.where(Jt < 0, 1, 2))) >= 0))


@pytest.mark.parametrize("kind,nl", [("A", 1), ("A", 2), ("A", 5), ("A", 20), ("B", 3), ("B", 16),
                                     ("A", 121)])
def test_factorization_reproduces_t(kind, nl):
    for a in range(2):
        T, _, _ = atom(kind, nl, a=a)
        Mt, Jt, perm, ex = P1.hebpj(T)
        assert factor_ok(T, Mt, Jt)
        check_pivots(T, perm, ex["blocks"])


def test_indefinite_blocks_take_2x2_pivots():
    # a zero diagonal forces order-2 pivots
    rng = np.random.default_rng(3)
    X = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    T = X + X.conj().T
    np.fill_diagonal(T, 0.0)
    Mt, Jt, perm, ex = P1.hebpj(T)
    assert any(s == 2 for _, s in ex["blocks"])
    assert factor_ok(T, Mt, Jt)
    check_pivots(T, perm, ex["blocks"])


def test_closed_forms():
    Mt, Jt, perm, ex = P1.hebpj(np.diag([3.0, -5.0, 1.0]).astype(complex))
    # pivots by decreasing |d|: -5 (index 1), 3 (index 0), 1 (index 2); positives first
    assert list(perm) == [1, 0, 2]
    assert list(Jt) == [1, 1, -1]
    np.testing.assert_allclose(Mt, [[math.sqrt(3), 0, 0], [0, 0, 1], [0, math.sqrt(5), 0]],
                               atol=1e-15)
    Mt, Jt, perm, ex = P1.hebpj(np.array([[0, 2], [2, 0]], dtype=complex))
    assert ex["blocks"] == [(0, 2)]
    assert list(Jt) == [1, -1]
    np.testing.assert_allclose(Mt, [[1, 1], [1, -1]], atol=1e-15)


def test_singular_t_leaves_zero_signs():
    # rank 2: the Schur complement after two pivots is exactly zero
    v = np.array([1.0, 2.0, 0.0, 1.0])
    w = np.array([0.0, 1.0, 1.0, 3.0])
    T = (np.outer(v, v) - np.outer(w, w)).astype(complex)
    Mt, Jt, perm, ex = P1.hebpj(T)
    assert ex["blocks"][-1][1] == 0
    assert list(Jt).count(0) == 2 and Jt[-1] == 0 and Jt[-2] == 0
    assert np.abs(Mt[-2:]).max() == 0.0
    assert factor_ok(T, Mt, Jt)
    Mt, Jt, perm, ex = P1.hebpj(np.zeros((3, 3), dtype=complex))
    assert list(Jt) == [0, 0, 0] and np.abs(Mt).max() == 0.0


def assembly_ok(T, H, U, F, J, G):
    r, _, na = T.shape
    nl = r // 2
    Href = sum(H[a * r:(a + 1) * r].conj().T @ T[:, :, a] @ H[a * r:(a + 1) * r]
               for a in range(na))
    S = 0
    for a in range(na):
        Ha = H[a * r:(a + 1) * r]
        Sa = np.vstack([Ha[:nl], U[:, a][:, None] * Ha[nl:]])
        S = S + Sa.conj().T @ Sa
    Hf = F.conj().T @ (J.astype(float)[:, None] * F)
    return (np.abs(Hf - Href).max() <= 1e-12 * np.abs(Href).max() and
            np.abs(G.conj().T @ G - S).max() <= 1e-12 * np.abs(S).max())


@pytest.mark.parametrize("kind", ["A", "B"])
def test_assembly_invariants(kind):
    T, H, U = synth.phase1_set(11, 5, kind, 6, 30)
    F, J, G, info = P1.phase1(T, H, U)
    assert assembly_ok(T, H, U, F, J, G)
    assert J.shape == (H.shape[0],) and set(np.unique(J)) <= {-1, 1}


def test_end_to_end_eigenvalues_match_scipy():
    # (F~, J~, G~) through the HZ oracle give the eigenvalues of (H, S)
    T, H, U = synth.phase1_set(12, 4, "A", 5, 24)
    F, J, G, _ = P1.phase1(T, H, U)
    Hm = F.conj().T @ (J.astype(float)[:, None] * F)
    Sm = G.conj().T @ G
    ref = np.sort(sla.eigh(Hm, Sm, eigvals_only=True))
    st, lam, X, stats = O.Oracle().ghsvd(F, J.astype(np.int8), G, reduce=True, order=0,
                                         max_sweeps=60)
    assert st == 0
    np.testing.assert_allclose(np.sort(lam), ref, rtol=1e-10, atol=0)


def battery():
    fails = []
    for kind, nl in (("A", 5), ("B", 4)):
        T, _, _ = atom(kind, nl, a=1)
        Mt, Jt, perm, ex = P1.hebpj(T)
        if not factor_ok(T, Mt, Jt):
            fails.append("factor")
        try:
            check_pivots(T, perm, ex["blocks"])
        except AssertionError:
            fails.append("pivots")
    rng = np.random.default_rng(5)
    X = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    T = X + X.conj().T
    np.fill_diagonal(T, 0.0)
    Mt, Jt, perm, ex = P1.hebpj(T)
    if not factor_ok(T, Mt, Jt):
        fails.append("factor2x2")
    T, H, U = synth.phase1_set(13, 3, "A", 4, 12)
    F, J, G, _ = P1.phase1(T, H, U)
    if not assembly_ok(T, H, U, F, J, G):
        fails.append("assembly")
    return fails


@pytest.mark.parametrize("mutant", range(1, 7))
def test_planted_mistakes_are_caught(mutant, monkeypatch):
    assert battery() == []
    monkeypatch.setattr(P1, "MUTANT", mutant)
    assert battery() != [], f"mutant {mutant} not caught"
