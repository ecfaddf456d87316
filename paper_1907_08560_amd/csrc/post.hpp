// post.hpp -- outputs of the sweeps (lambda, X).
#pragma once

#include "hz_common.hpp"

namespace ghsvd {

// lambda[rank_j] = h_j / s_j, X(perm[i], rank_j) = Z(i, j) / sqrt(s_j).
// flags[0] |= 1 when G is numerically rank deficient (a vanishing s_j, or
// ||x_j|| ||G||_F >= 1 / (sqrt(n) eps)), |= 2 for non-finite values.
// perm may be NULL (identity).  Scratch: lam_tmp, scale (n doubles), rank (n ints).
int postprocess(int m, int nplus, int p, int n, const double2 *F, long ldf, const double2 *G,
                long ldg, const double2 *Z, long ldz, const int *perm, const double *gnorm2,
                int sort, double *lam_tmp, double *scale, int *rank, int *flags, double *lambda,
                double2 *X, long ldx, hipStream_t stream);

}  // namespace ghsvd
