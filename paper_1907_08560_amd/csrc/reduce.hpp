// reduce.hpp -- one-time reduction to square factors (Section 5) and the
// signature split (Section 4.5.1 form with one negative block).
#pragma once

#include "hz_common.hpp"

namespace ghsvd {

// Device state of the hyperbolic QR; the column loop is driven from the
// device (each kernel reads it), so the host enqueues a fixed sequence.
struct JqrState {
    int k;       // first unreduced column (and row)
    int piv;     // 1 or 2: pivot size chosen for column k
    int need2;   // Bunch-Kaufman second test required
    int ii;      // Bunch-Kaufman candidate column
    int status;  // 0 or an error
    int n2x2;    // 2x2 pivots taken
    int pad[2];
    double lam;  // |h_{k,ii}|
    double tau[2];
    double co, si;
    double2 eph;
};

struct JqrBufs {
    JqrState *st;
    double *hd;   // [n] J-norms of the trailing columns
    double2 *hc;  // [n] J-products with the pivot column
    double *hi;   // [n] |J-products| with the candidate column
    double2 *s;   // [2 * m] reflector generators
};

// Hyperbolic QR of A (m x n, lda) in place under the signature J (m int8,
// permuted in place).  perm (n ints) receives P2.  Synchronizes the stream
// once at the end; returns the status, *n2x2 the 2x2 pivot count.
int run_jqr(int m, int n, double2 *A, long lda, int8_t *J, int *perm, const JqrBufs &b,
            hipStream_t stream, int *n2x2);

// Householder QR of A (p x n, lda) in place: R in the upper triangle, zeros
// below; R_kk = -e^{i arg x_1} ||x||.  v: p complex scratch, coef: 1 double.
int run_qr(int p, int n, double2 *A, long lda, double2 *v, double *coef, hipStream_t stream);

// dst(:, j) = src(:, perm[j]) for rows 0..rows-1 (perm may be NULL = identity).
int copy_cols(int rows, int n, const double2 *src, long lds, double2 *dst, long ldd,
              const int *perm, hipStream_t stream);

// Stable row partition by sign: rows with J = +1 first.  Rows 0..rows-1 of
// src (n columns) go to dst; *nplus_dev receives the count of +1 rows.
// rowmap: rows ints scratch.
int jsplit(int rows, int n, const double2 *src, long lds, const int8_t *J, double2 *dst,
           long ldd, int *rowmap, int *nplus_dev, hipStream_t stream);

// Checks the inputs: J entries in {+1, -1}, F and G finite; accumulates
// ||G||_F^2 into gnorm2[0].  flags[0] |= 1 (bad J), 2 (non-finite).
int check_inputs(int m, int n, int p, const double2 *F, long ldf, const int8_t *J,
                 const double2 *G, long ldg, int *flags, double *gnorm2, hipStream_t stream);

// Identity matrix n x n (ld) of complex128 or complex64.
int set_identity(int n, void *Z, long ldz, int fp32, hipStream_t stream);

}  // namespace ghsvd
