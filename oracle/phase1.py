"""Phase 1: simultaneous factorizations of the atom blocks T_a -- TEST INFRASTRUCTURE.

Only the test suite and the benchmark may import this module; the solver
never does.  Plain numpy, FP64, written from the paper (Section 4):

* `bunch_parlett`: the Hermitian indefinite factorization T = P^T M^* D M P
  of Section 4.2 with the complete pivoting of Bunch and Parlett: M upper
  triangular with identity diagonal blocks, D block diagonal with blocks of
  order 1 or 2, P a permutation;
* `hebpj`: ZHEBPJ, i.e. that factorization followed by the transformation
  of D into J^ = diag(+-1) (Section 4.2: a block of order 1 scales its row
  of M by |d|^{1/2}; a block of order 2 is diagonalized by a Jacobi rotation
  R_k, its two rows of M are multiplied by R_k^*, then scaled the same way),
  the postprocessing M^ = M P and the inner permutation that puts the
  positive signs first (Section 4.3): T = M~^* J~ M~;
* `phase1`: the per-atom loop of Section 4.4 (factor T_a, F~_a = M~_a H_a,
  G~_a = [A_a; U_a B_a]) assembling F~, J~, G~ of Section 4.1-4.3 (eq. (4.1),
  (4.2)).

Readings where the paper is silent:
  * The pivot test uses the Bunch-Parlett constant alpha = (1 + sqrt(17)) / 8
    and compares squared moduli, mu1^2 >= alpha^2 mu0^2, where mu0 is the
    largest modulus in the remaining Schur complement and mu1 the largest
    diagonal modulus.  Only the upper triangle (i <= j) of the Schur
    complement is read, and only the real part of its diagonal; moduli are
    re^2 + im^2.
  * Ties: a 1x1 pivot is the first maximal diagonal entry; a 2x2 pivot is
    the first maximal strictly-upper entry (i, j) in column-major order
    (smallest j, then smallest i), and i takes the earlier position.
  * The Jacobi rotation of a 2x2 block [[a, c], [conj(c), b]] is the
    symmetric Schur rotation applied after the phase of c is moved out:
    tau = (b - a) / (2 |c|), t = sign(tau) / (|tau| + sqrt(1 + tau^2))
    (sign(0) = +1), cs = (1 + t^2)^{-1/2}, sn = t cs; with e = c / |c|,
    R = [[cs, sn], [-sn conj(e), cs conj(e)]] and R^* E R =
    diag(a - t |c|, b + t |c|).
  * A Schur complement that is exactly zero ends the factorization; its
    remaining rows of M~ are zero and their signs 0, placed last.
  * The inner permutation is stable: within each sign the rows keep the
    order in which the factorization produced them.

Mutation switch: MUTANT (module level, 0 = none) plants one mistake for the
pin tests: 1 pivot test without alpha, 2 conjugate dropped in the Schur
update of a 1x1 pivot, 3 rotation applied untransposed, 4 row scaling by
|d| instead of |d|^{1/2}, 5 positives not put first, 6 B_a rows left unscaled.
"""
from __future__ import annotations

import math

import numpy as np

MUTANT = 0
ALPHA = (1.0 + math.sqrt(17.0)) / 8.0


def _mod2(z):
    return np.real(z) * np.real(z) + np.imag(z) * np.imag(z)


def bunch_parlett(T):
    """Section 4.2: T = P^T M^* D M P by Bunch-Parlett complete pivoting.

    Returns (M, D, perm, blocks):
      M      r x r complex, upper triangular in the pivoted order, identity on
             the diagonal blocks (rows of a zero tail are zero);
      D      r x r complex, block diagonal (blocks of order 1 or 2);
      perm   perm[k] = the index of T that sits at pivoted position k
             (P T P^T = T[perm][:, perm]);
      blocks list of (k, s): a pivot block of order s at position k, s = 0 for
             the zero tail starting at k.
    """
    A = np.array(T, dtype=np.complex128, copy=True)
    r = A.shape[0]
    perm = np.arange(r)
    M = np.zeros((r, r), dtype=np.complex128)
    D = np.zeros((r, r), dtype=np.complex128)
    blocks = []
    k = 0
    a2 = ALPHA * ALPHA
    while k < r:
        S = A[k:, k:]
        rr = r - k
        diag2 = np.real(np.diagonal(S)) ** 2
        mu1 = float(diag2.max())
        iu = np.triu_indices(rr, 1)
        off2 = _mod2(S[iu]) if rr > 1 else np.zeros(0)
        mu0 = max(mu1, float(off2.max()) if off2.size else 0.0)
        if mu0 == 0.0:
            blocks.append((k, 0))
            break
        one = mu1 >= (mu0 if MUTANT == 1 else a2 * mu0)
        if one:
            i = k + int(np.argmax(diag2))
            piv = [i]
        else:
            # first maximum in column-major order over the strict upper triangle
            cols, rows = iu[1], iu[0]
            order = np.lexsort((rows, cols))
            best = order[int(np.argmax(off2[order]))]
            piv = [k + int(rows[best]), k + int(cols[best])]
        # symmetric interchanges: the chosen indices move to positions k, k+1
        for t, src in enumerate(piv):
            dst = k + t
            if src != dst:
                A[[dst, src], :] = A[[src, dst], :]
                A[:, [dst, src]] = A[:, [src, dst]]
                M[:, [dst, src]] = M[:, [src, dst]]  # the rows already formed
                perm[[dst, src]] = perm[[src, dst]]
                # a later chosen index that sat at dst now sits at src
                piv = [src if (q == dst and u > t) else q for u, q in enumerate(piv)]
        s = len(piv)
        E = A[k:k + s, k:k + s].copy()
        for t in range(s):
            E[t, t] = np.real(E[t, t])
        if s == 2:
            E[1, 0] = np.conj(E[0, 1])
        B = A[k:k + s, k + s:]
        Einv = np.linalg.inv(E)
        M[k:k + s, k:k + s] = np.eye(s)
        M[k:k + s, k + s:] = Einv @ B
        D[k:k + s, k:k + s] = E
        if s == 1 and MUTANT == 2:
            A[k + 1:, k + 1:] -= np.outer(B[0], B[0]) / np.real(E[0, 0])
        else:
            A[k + s:, k + s:] -= B.conj().T @ (Einv @ B)
        blocks.append((k, s))
        k += s
    return M, D, perm, blocks


def jacobi_2x2(E):
    """The rotation R with R^* E R = diag(l1, l2) for a Hermitian 2x2 block E
    (see the module header).  Returns (R, l1, l2)."""
    a = float(np.real(E[0, 0]))
    b = float(np.real(E[1, 1]))
    c = complex(E[0, 1])
    ac = abs(c)
    if ac == 0.0:
        return np.eye(2, dtype=np.complex128), a, b
    tau = (b - a) / (2.0 * ac)
    t = (1.0 if tau >= 0.0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
    cs = 1.0 / math.sqrt(1.0 + t * t)
    sn = t * cs
    e = c / ac
    R = np.array([[cs, sn], [-sn * np.conj(e), cs * np.conj(e)]], dtype=np.complex128)
    return R, a - t * ac, b + t * ac


def hebpj(T):
    """ZHEBPJ (Sections 4.2, 4.3): T = Mt^* diag(Jt) Mt.

    Returns (Mt, Jt, perm, blocks): Mt r x r complex, Jt r int8 (+1 first,
    then -1, then 0), perm and blocks as `bunch_parlett`; `order[i]` of the
    extra dict entry gives the factor row (pivoted position) that became row
    i of Mt."""
    M, D, perm, blocks = bunch_parlett(T)
    r = M.shape[0]
    Jh = np.zeros(r, dtype=np.int8)
    for k, s in blocks:
        if s == 0:
            M[k:, :] = 0.0
            break
        if s == 1:
            d = float(np.real(D[k, k]))
            Jh[k] = 1 if d > 0.0 else -1
            M[k, :] *= abs(d) if MUTANT == 4 else math.sqrt(abs(d))
        else:
            R, l1, l2 = jacobi_2x2(D[k:k + 2, k:k + 2])
            rows = (R if MUTANT == 3 else R.conj().T) @ M[k:k + 2, :]
            Jh[k] = 1 if l1 > 0.0 else -1
            Jh[k + 1] = 1 if l2 > 0.0 else -1
            M[k, :] = math.sqrt(abs(l1)) * rows[0]
            M[k + 1, :] = math.sqrt(abs(l2)) * rows[1]
    # M^ = M P: column k of M belongs to column perm[k] of T
    Mh = np.zeros_like(M)
    Mh[:, perm] = M
    # inner permutation: positive signs first, then negative, then zero
    if MUTANT == 5:
        order = np.arange(r)
    else:
        order = np.concatenate([np.nonzero(Jh == 1)[0], np.nonzero(Jh == -1)[0],
                                np.nonzero(Jh == 0)[0]])
    return Mh[order], Jh[order], perm, {"blocks": blocks, "order": order}


def phase1(T, H, U):
    """Section 4.4, the per-atom loop: for every atom a, T_a = Mt_a^* Jt_a Mt_a,
    F~_a = Mt_a H_a, G~_a = [A_a; U_a B_a].

    T  r x r x N_A complex (T[:, :, a] = T_a, r = 2 N_L);
    H  (r N_A) x n complex, rows a r .. a r + r - 1 = H_a = [A_a; B_a];
    U  N_L x N_A real, column a = the diagonal of U_a.
    Returns (F, J, G, info): F, G (r N_A) x n complex, J (r N_A) int8, info a
    list of the per-atom (perm, blocks)."""
    r, _, na = T.shape
    nl = r // 2
    m, n = H.shape
    F = np.zeros((m, n), dtype=np.complex128, order="F")
    G = np.zeros((m, n), dtype=np.complex128, order="F")
    J = np.zeros(m, dtype=np.int8)
    info = []
    for a in range(na):
        Mt, Jt, perm, ex = hebpj(T[:, :, a])
        Ha = H[a * r:(a + 1) * r, :]
        F[a * r:(a + 1) * r, :] = Mt @ Ha
        J[a * r:(a + 1) * r] = Jt
        G[a * r:a * r + nl, :] = Ha[:nl, :]
        scale = np.ones(nl) if MUTANT == 6 else U[:, a]
        G[a * r + nl:(a + 1) * r, :] = scale[:, None] * Ha[nl:, :]
        info.append((perm, ex["blocks"]))
    return F, J, G, info
