"""The explicit-formation alternative (Section 4.5) -- TEST INFRASTRUCTURE.

Only the test suite and the benchmark may import this module; the solver
never does.  Plain numpy / scipy, FP64.  Section 4.5 forms the pencil
explicitly, S = G^* G (one Hermitian rank-k product) and H = F^* J F (the rows
of a copy of F scaled by J, then one product), and hands (H, S) to a
Cholesky-based generalized Hermitian eigensolver (ZHEGV / ZHEGVD):

  * `form`: H and S as above;
  * `solve_explicit`: S = R^* R (Cholesky, R upper triangular with a positive
    real diagonal), C = R^{-*} H R^{-1}, C = Y diag(lambda) Y^* (a Hermitian
    eigensolver of the library), X = R^{-1} Y, eigenvalues ascending.  Then
    H X = S X diag(lambda) and X^* S X = I, the normalization of eq. (3.2).

The route squares the conditioning of G: its eigenvalues carry a relative
error of order eps cond(S), which is why the paper keeps the implicit HZ
method for ill-conditioned S.  Nothing here is blocked or reordered beyond
the library calls.

Mutation switch: MUTANT (module level, 0 = none): 1 J dropped from H, 2 the
reduction taken as R^{-1} H R^{-*}, 3 X = R^{-*} Y, 4 descending order.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

MUTANT = 0


def form(F, J, G):
    """Section 4.5: H = F^* J F (J applied to the rows of a copy of F) and
    S = G^* G."""
    F = np.asarray(F, dtype=np.complex128)
    G = np.asarray(G, dtype=np.complex128)
    j = np.ones(F.shape[0]) if MUTANT == 1 else np.asarray(J, dtype=np.float64)
    H = F.conj().T @ (j[:, None] * F)
    S = G.conj().T @ G
    return H, S


def solve_explicit(F, J, G):
    """(lambda, X, R, C) of the explicitly formed pencil (see the header).
    Raises numpy.linalg.LinAlgError when S is not numerically positive
    definite."""
    H, S = form(F, J, G)
    R = np.linalg.cholesky(S).conj().T  # S = R^* R, R upper
    if MUTANT == 2:
        W = sla.solve_triangular(R, H, lower=False)
        C = sla.solve_triangular(R, W.conj().T, lower=False).conj().T
    else:
        W = sla.solve_triangular(R, H, trans="C", lower=False)           # R^{-*} H
        C = sla.solve_triangular(R, W.conj().T, trans="C", lower=False)  # R^{-*} (R^{-*} H)^*
    C = 0.5 * (C + C.conj().T)
    lam, Y = np.linalg.eigh(C)
    if MUTANT == 3:
        X = sla.solve_triangular(R, Y, trans="C", lower=False)
    else:
        X = sla.solve_triangular(R, Y, lower=False)
    order = np.argsort(-lam if MUTANT == 4 else lam, kind="stable")
    return lam[order], X[:, order], R, C
