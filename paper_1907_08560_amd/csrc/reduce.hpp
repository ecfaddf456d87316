// reduce.hpp -- one-time reduction to square factors (Section 5) and the
// signature split (Section 4.5.1 form with one negative block).
#pragma once

#include <vector>

#include "batch.hpp"
#include "sweep.hpp"

namespace ghsvd {

// Hyperbolic QR of every pencil's Ft (m x n) under Jw, in place, with P2 in
// perm; and the Householder QR of Gt = G without pivoting (R_kk = -e^{i arg
// x_1} ||x||; the caller permutes R's columns by P2).  Pencils with reduce =
// 0 are skipped.  One launch per step covers all pencils.  Synchronizes the
// stream; status[k] and n2x2[k] per pencil.
int run_reduction(BatchCtx &c, std::vector<int> &status, std::vector<int> &n2x2,
                  hipStream_t s);

// dst(:, j) = src(:, perm[j]) for rows 0..rows-1 (perm may be NULL = identity).
int copy_cols(int rows, int n, const double2 *src, long lds, double2 *dst, long ldd,
              const int *perm, hipStream_t stream);

// Stable row partition by sign: rows with J = +1 first.  Rows 0..rows-1 of
// src (n columns) go to dst; *nplus_dev receives the count of +1 rows.
int jsplit(int rows, int n, const double2 *src, long lds, const int8_t *J, double2 *dst,
           long ldd, int *rowmap, int *nplus_dev, hipStream_t stream);

// Checks the inputs: J entries in {+1, -1}, F and G finite; writes
// ||G||_F^2 into gnorm2[0], summed in a fixed order from per-workgroup
// partials kept in gnorm2[1 .. 8 n] (the buffer holds 1 + 8 n doubles).
// flags[0] |= 1 (bad J), 2 (non-finite).
int check_inputs(int m, int n, int p, const double2 *F, long ldf, const int8_t *J,
                 const double2 *G, long ldg, int *flags, double *gnorm2, hipStream_t stream);

// Row map of the split alone (rowmap, *nplus_dev), for jqr_extract.
int jsplit_map(int rows, const int8_t *J, int *rowmap, int *nplus_dev, hipStream_t stream);

// F_sq (n x n, columns in the order of P2) of a reduced pencil from its
// factored columns into dst (ld ldd), rows moved by rowmap (NULL: in place);
// scatter = 1 puts column j of the factor at column perm[j] instead (the
// input's column order).
int jqr_extract(const PencilDev &P, double2 *dst, long ldd, const int *rowmap, hipStream_t stream,
                int scatter = 0);

// Identity matrix n x n (ld) of complex128 or complex64.
int set_identity(int n, void *Z, long ldz, int fp32, hipStream_t stream);

}  // namespace ghsvd
