"""Full GHSVD from a converged sweep stage (Phase 4) -- TEST INFRASTRUCTURE.

Only the test suite and the benchmark may import this module; the solver
never does.  Plain numpy, FP64, written from the paper:

* `outputs`: the outputs of the implicit HZ algorithm (Section 6.1,
  paragraph "Outputs"): Sigma_F' = diag(|f_j^* J f_j|^{1/2}), Sigma_G' =
  diag(||g_j||), U = F' Sigma_F'^{-1}, V = G' Sigma_G'^{-1}, Sigma_j =
  ((Sigma_F')_j^2 + (Sigma_G')_j^2)^{1/2}, Sigma_F = Sigma_F' Sigma^{-1},
  Sigma_G = Sigma_G' Sigma^{-1}, Z = Z' Sigma^{-1};
* `lu_complete`: the LU factorization with complete pivoting of Section 7
  (P A Q = L U, L unit lower triangular);
* `inverse_from_lu`: X = Z^{-1} from that factorization, column by column
  (Section 7 solves Z X = I);
* `full_ghsvd`: the above in sequence, F' = U Sigma_F X, G' = V Sigma_G X;
* `decomposition_errors`: the relative errors (7.1).

Reading where the paper is silent: among entries of equal modulus the pivot
is the first in column-major order (smallest column, then smallest row).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def outputs(Fp, J, Gp, Zp):
    """Section 6.1, "Outputs": (U, V, sigma_f, sigma_g, Z) from the swept F', G'
    and the accumulated transformation Z'.  sigma_f, sigma_g are the diagonals
    of Sigma_F and Sigma_G."""
    Fp = np.asarray(Fp, dtype=np.complex128)
    Gp = np.asarray(Gp, dtype=np.complex128)
    Zp = np.asarray(Zp, dtype=np.complex128)
    j = np.asarray(J, dtype=np.float64)
    hj = np.real(np.sum(np.conj(Fp) * (j[:, None] * Fp), axis=0))  # f_j^* J f_j
    gj = np.real(np.sum(np.conj(Gp) * Gp, axis=0))                  # g_j^* g_j
    sf = np.sqrt(np.abs(hj))
    sg = np.sqrt(gj)
    sig = np.sqrt(sf * sf + sg * sg)
    U = Fp / sf[None, :]
    V = Gp / sg[None, :]
    return U, V, sf / sig, sg / sig, Zp / sig[None, :]


def lu_complete(A):
    """Section 7: P A Q = L U with complete pivoting.  Returns (LU, rows, cols):
    LU holds L below the diagonal (unit diagonal implied) and U on and above
    it; row i of P A is row rows[i] of A, column j of A Q is column cols[j]."""
    LU = np.array(A, dtype=np.complex128, copy=True)
    n = LU.shape[0]
    rows = np.arange(n)
    cols = np.arange(n)
    for k in range(n):
        mod = np.abs(LU[k:, k:])
        # first maximum in column-major order
        flat = np.argmax(mod.T.reshape(-1))
        q, p = divmod(int(flat), n - k)
        p += k
        q += k
        if mod[p - k, q - k] == 0.0:
            raise ZeroDivisionError("singular matrix")
        LU[[k, p], :] = LU[[p, k], :]
        rows[[k, p]] = rows[[p, k]]
        LU[:, [k, q]] = LU[:, [q, k]]
        cols[[k, q]] = cols[[q, k]]
        if k + 1 < n:
            LU[k + 1:, k] /= LU[k, k]
            LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, rows, cols


def inverse_from_lu(LU, rows, cols):
    """A^{-1} from P A Q = L U: A^{-1} = Q U^{-1} L^{-1} P."""
    n = LU.shape[0]
    P = np.eye(n, dtype=np.complex128)[rows, :]          # P A = A[rows, :]
    Y = sla.solve_triangular(LU, P, lower=True, unit_diagonal=True)
    W = sla.solve_triangular(LU, Y, lower=False)
    X = np.empty_like(W)
    X[cols, :] = W                                          # Q W
    return X


def full_ghsvd(Fp, J, Gp, Zp):
    """(U, V, sigma_f, sigma_g, X) with F' Z'^{-1} = U Sigma_F X and
    G' Z'^{-1} = V Sigma_G X (the swept factors' starting matrices)."""
    U, V, sf, sg, Z = outputs(Fp, J, Gp, Zp)
    LU, rows, cols = lu_complete(Z)
    return U, V, sf, sg, inverse_from_lu(LU, rows, cols)


def decomposition_errors(F, G, U, V, sigma_f, sigma_g, X):
    """Eq. (7.1): ||F - U Sigma_F X||_F / ||F||_F and ||G - V Sigma_G X||_F / ||G||_F."""
    eF = np.linalg.norm(F - (U * sigma_f[None, :]) @ X) / np.linalg.norm(F)
    eG = np.linalg.norm(G - (V * sigma_g[None, :]) @ X) / np.linalg.norm(G)
    return float(eF), float(eG)
