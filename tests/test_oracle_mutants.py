"""Planted mistakes in the oracle must be caught by its pins.

hz_oracle.c carries compile-time switches ORA_MUTANT = 1..16, each a
plausible slip (a sign, a conjugate, a transposed operand, a dropped scaling,
a wrong index, a skipped pivoting rule).  This test builds each variant on the
CPU and runs a compact battery of the same independent checks the pin tests
use; every variant must fail at least one of them, and the unmutated build
must pass all of them.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_08560_amd import synth

EPS = 2.0 ** -52
MUTANTS = list(range(1, 17))


def battery(o):
    """Returns the names of the checks that fail for oracle `o`."""
    fails = []
    # pair: diagonalization of random well-conditioned 2x2 pencils
    d = synth.random_pairs(101, 60)
    for i in range(60):
        a, b, c, sa, sb, sc = (d[k][i] for k in ("a", "b", "c", "sa", "sb", "sc"))
        x = abs(sc) / math.sqrt(sa * sb)
        if x > 0.9:
            continue
        kind, Z = o.pair_params(a, b, c, sa, sb, sc, EPS * 8)
        H = np.array([[a, c], [np.conj(c), b]])
        S = np.array([[sa, sc], [np.conj(sc), sb]])
        MS = Z.conj().T @ S @ Z
        MH = Z.conj().T @ H @ Z
        if kind <= 0 or np.abs(MS - np.eye(2)).max() > 1e-10 or \
                abs(MH[0, 1]) > 1e-10 * np.abs(np.diag(MH)).max():
            fails.append("pair")
            break
    # ordering coverage
    for n in (8, 9):
        steps, pp, qq = o.round_robin(n)
        pairs = {(int(p), int(q)) for p, q in zip(pp.ravel(), qq.ravel()) if p >= 0}
        if len(pairs) != n * (n - 1) // 2:
            fails.append("order")
    # QR against the library up to phases
    P = synth.random_pencil(102, 12, 18, 13, 24, 1e-3)
    st, R = o.qr(P.G)
    r = np.linalg.qr(P.G)[1]
    if st != 0 or np.abs(np.abs(R) - np.abs(r)).max() > 1e-12:
        fails.append("qr")
    # JQR invariant
    st, Fsq, Jsq, perm, n2, A = o.jqr(P.F, P.J)
    H = P.F.conj().T @ (P.J[:, None] * P.F)
    if st != 0 or np.abs(Fsq.conj().T @ (Jsq[:, None] * Fsq) - H[np.ix_(perm, perm)]).max() \
            > 1e-12 * np.abs(H).max():
        fails.append("jqr")
    # 2x2 pivot forced by J-isotropic columns
    F2 = np.zeros((6, 2), dtype=complex)
    J2 = np.array([1, 1, 1, -1, -1, -1])
    F2[0, 0] = F2[3, 0] = 1.0
    F2[1, 1] = F2[4, 1] = 1.0
    F2[0, 1], F2[3, 1] = 2.0, -2.0
    st, Fs2, Js2, perm2, n22, _ = o.jqr(F2, J2)
    H2 = F2.conj().T @ (J2[:, None] * F2)
    if st != 0 or n22 != 1 or \
            np.abs(Fs2.conj().T @ (Js2[:, None] * Fs2) - H2[np.ix_(perm2, perm2)]).max() > 1e-13:
        fails.append("jqr2x2")
    # order one: lambda = a / s_a, |x| = s_a^(-1/2)
    st, lam1, X1, _ = o.ghsvd(np.array([[1.0 + 2j], [3.0 - 1j]]), np.array([1, -1]),
                              np.array([[2.0 + 0j], [1j]]))
    if st != 0 or abs(lam1[0] - (-5.0 / 5.0)) > 1e-15 or abs(abs(X1[0, 0]) - 5 ** -0.5) > 1e-15:
        fails.append("order1")
    # whole solve against scipy at good conditioning, and invariants on factors
    import scipy.linalg as sl
    S = P.G.conj().T @ P.G
    ref = sl.eigh(H, S, eigvals_only=True)
    for reduce in (False, True):
        st, lam, X, stats = o.ghsvd(P.F, P.J, P.G, reduce=reduce, order=1)
        if st < 0 or np.max(np.abs(lam - ref) / np.abs(ref)) > 1e-9:
            fails.append(f"solve{int(reduce)}")
            continue
        GX = P.G @ X
        FX = P.F @ X
        Hx = FX.conj().T @ (P.J[:, None] * FX)
        if np.abs(GX.conj().T @ GX - np.eye(P.n)).max() > 1e-9 or \
                np.abs(np.real(np.diag(Hx)) - lam).max() > 1e-9 * np.abs(lam).max():
            fails.append(f"inv{int(reduce)}")
    # Full Block inner level on a pencil of one block pair: Algorithm 2 with
    # its own stopping test (no transformation) on the (J)QR-shortened pivot
    Q = synth.random_pencil(103, 16, 24, 18, 32, 1e-2)
    st, Fb, Gb, Zb, sb = o.hz_block_run(Q.F, Q.J, Q.G, w=8, max_sweeps=1, inner_order=2)
    st_, A, Jh, perm, _, _ = o.jqr(Q.F, Q.J)
    st2, R = o.qr(np.asfortranarray(Q.G[:, perm]))
    Ft = np.zeros((16, 16), dtype=complex)
    Gt = np.zeros((16, 16), dtype=complex)
    Ft[:, perm] = A
    Gt[:, perm] = R
    st3, _, _, _, s3 = o.hz_run(np.asfortranarray(Ft), Jh, np.asfortranarray(Gt), order=1,
                                max_sweeps=30, stop_rule=1)
    if st < 0 or st3 != 0 or sb[1] != s3[1]:
        fails.append("fb")
    # three-level BO on a pencil of one block pair (n = 32, w = 16): one nested
    # blocked sweep of width 8 over the shortened pivot, 3 block steps of 2
    # block pivots of 16 columns (120 pairs each)
    Q = synth.random_pencil(105, 32, 48, 36, 64, 1e-2)
    st, Fb, Gb, Zb, sb = o.hz_block_run(Q.F, Q.J, Q.G, w=16, max_sweeps=1, inner_order=3)
    if st < 0 or sb[1] != 3 * 2 * 120:
        fails.append("ml")
    return fails


def test_unmutated_passes_battery(oracle):
    assert battery(oracle) == []


@pytest.mark.parametrize("k", MUTANTS)
def test_mutant_is_caught(k):
    path = O.build(mutant=k)
    try:
        o = O.Oracle(path)
        fails = battery(o)
    finally:
        import os
        os.remove(path)
    assert fails, f"planted mistake {k} passed every pin"
