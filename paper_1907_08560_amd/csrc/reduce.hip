// reduce.hip -- one-time reduction of tall F, G to square factors (Section 5).
//
// F: hyperbolic QR (JQR, eq. (5.1)) with diagonal pivoting supplemented by
// Bunch-Kaufman partial pivoting (Section 5.2.1, alpha = (1 + sqrt(17)) / 8),
// single pivots reduced by the hyperbolic Householder reflector H(s) of
// Section 5.3 (Theorem 5.1, generator s = f + c_1 e_1 with arg c_1 = arg f_11,
// a matching-sign row swapped to the front when needed), 2x2 pivots by the
// (J, I) URV step (Jacobi rotation of the pivot J-Gram, two reflectors, R^*).
// G: Householder QR of G P2 (the "TSQR" step; Q is not formed).
//
// The k-loop of the JQR is sequential; each iteration is a fixed sequence of
// kernels that read the iteration's state from device memory (pivot size,
// candidate column), so no host round trip is needed per column.  Kernels
// over all trailing columns use one workgroup per column (column-major, rows
// read coalesced); decisions run in a single 1024-thread workgroup.
#include "reduce.hpp"

namespace ghsvd {

constexpr int kGridNT = 256;
constexpr int kOneNT = 1024;

__device__ __forceinline__ double jsign(const int8_t *J, int r) { return (double)J[r]; }

// Block-wide J-weighted dot conj(x)^T diag(J) y over rows r0..m-1.
__device__ __forceinline__ double2 jdot_block(const double2 *x, const double2 *y, const int8_t *J,
                                              int r0, int m, double *red) {
    double v[2] = {0.0, 0.0};
    for (int r = r0 + threadIdx.x; r < m; r += blockDim.x) {
        const double s = jsign(J, r);
        const double2 a = x[r], b = y[r];
        v[0] += s * (a.x * b.x + a.y * b.y);
        v[1] += s * (a.x * b.y - a.y * b.x);
    }
    block_sum<2>(v, red);
    return cmk(v[0], v[1]);
}

__device__ __forceinline__ double jnorm_block(const double2 *x, const int8_t *J, int r0, int m,
                                              double *red) {
    double v[1] = {0.0};
    for (int r = r0 + threadIdx.x; r < m; r += blockDim.x) v[0] += jsign(J, r) * cnorm2(x[r]);
    block_sum<1>(v, red);
    return v[0];
}

__device__ __forceinline__ void swap_cols_block(double2 *A, long lda, int m, int c1, int c2) {
    if (c1 == c2) return;
    double2 *x = A + (size_t)c1 * lda;
    double2 *y = A + (size_t)c2 * lda;
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        const double2 t = x[r];
        x[r] = y[r];
        y[r] = t;
    }
}

__device__ __forceinline__ bool jqr_active(const JqrState *st, int n) {
    return st->status == 0 && st->k < n;
}

// hd[j] = J-norm^2 of column j over rows k..m-1 (first iteration only; later
// iterations get it from the apply kernel).
// Batched launches over columns: workgroup -> (pencil, column j) through the
// prefix sums of the column counts; single-workgroup phases: one workgroup
// per pencil.  Each kernel reads the pencil's fields below.
#define JQR_PENCIL_COL()                                          \
    const int pk = find_pencil(pre, B, blockIdx.x);                \
    const PencilDev P = PD[pk];                                  \
    if (!P.reduce) return;                                        \
    double2 *A = P.Ft;                                            \
    const long lda = P.ldft;                                      \
    const int m = P.m, n = P.n;                                   \
    int8_t *J = P.Jw;                                             \
    JqrState *st = P.jst;                                         \
    const int j_local = blockIdx.x - pre[pk];                     \
    (void)J;                                                      \
    (void)j_local
#define JQR_PENCIL_ONE()                                          \
    const PencilDev P = PD[blockIdx.x];                          \
    if (!P.reduce) return;                                        \
    double2 *A = P.Ft;                                            \
    const long lda = P.ldft;                                      \
    const int m = P.m, n = P.n;                                   \
    int8_t *J = P.Jw;                                             \
    JqrState *st = P.jst;                                         \
    (void)J;                                                      \
    (void)m

__global__ __launch_bounds__(kGridNT) void k_jqr_colnorms(const PencilDev *PD, const int *pre, int B) {
    __shared__ double red[kGridNT / kWave];
    JQR_PENCIL_COL();
    double *hd = P.hd;
    if (!jqr_active(st, n)) return;
    const int k = st->k;
    const int j = j_local;
    if (j < k) return;
    const double h = jnorm_block(A + (size_t)j * lda, J, k, m, red);
    if (threadIdx.x == 0) hd[j] = h;
}

// Every workgroup finds the diagonal pivot jmax = argmax |hd[j]| (j >= k) and
// workgroup j computes the J-product of column jmax with column j, stored at
// the position column j takes after the swap k <-> jmax.
__global__ __launch_bounds__(kGridNT) void k_jqr_cross(const PencilDev *PD, const int *pre, int B) {
    __shared__ double red[2 * kGridNT / kWave];
    __shared__ double rv[kGridNT / kWave];
    __shared__ int ri[kGridNT / kWave];
    JQR_PENCIL_COL();
    const double *hd = P.hd;
    double2 *hc = P.hc;
    if (!jqr_active(st, n)) return;
    const int k = st->k;
    const int j = j_local;
    if (j < k || k == n - 1) return;
    double bv = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(hd[i]);
        if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
    }
    block_argmax(bv, bi, rv, ri);
    if (j == bi) return;
    const double2 d = jdot_block(A + (size_t)bi * lda, A + (size_t)j * lda, J, k, m, red);
    const int pos = (j == k) ? bi : j;
    if (threadIdx.x == 0) hc[pos] = d;
}

// Applies the diagonal pivot swap and the first Bunch-Kaufman test.
__global__ __launch_bounds__(kOneNT) void k_jqr_decide1(const PencilDev *PD) {
    __shared__ double rv[kOneNT / kWave];
    __shared__ int ri[kOneNT / kWave];
    JQR_PENCIL_ONE();
    double *hd = P.hd;
    const double2 *hc = P.hc;
    int *perm = P.perm;
    if (!jqr_active(st, n)) return;
    const int k = st->k;
    double bv = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(hd[i]);
        if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
    }
    block_argmax(bv, bi, rv, ri);
    swap_cols_block(A, lda, m, k, bi);
    // candidate ii = argmax_{j > k} |h_kj| (hc already in post-swap positions)
    double cv = -1.0;
    int ci = k + 1;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
        const double v = sqrt(cnorm2(hc[i]));
        if (v > cv || (v == cv && i < ci)) { cv = v; ci = i; }
    }
    block_argmax(cv, ci, rv, ri);
    if (threadIdx.x == 0) {
        if (bi != k) {
            const int t = perm[k]; perm[k] = perm[bi]; perm[bi] = t;
            const double h = hd[k]; hd[k] = hd[bi]; hd[bi] = h;
        }
        const double alpha = (1.0 + sqrt(17.0)) / 8.0;
        st->piv = 1;
        st->need2 = 0;
        if (k < n - 1) {
            st->ii = ci;
            st->lam = cv;
            if (!(fabs(hd[k]) >= alpha * cv)) st->need2 = 1;
        }
    }
}

// hi[l] = |J-product of the candidate column ii with column l| (l >= k, l != ii).
__global__ __launch_bounds__(kGridNT) void k_jqr_cross2(const PencilDev *PD, const int *pre, int B) {
    __shared__ double red[2 * kGridNT / kWave];
    JQR_PENCIL_COL();
    double *hi = P.hi;
    if (!jqr_active(st, n) || !st->need2) return;
    const int k = st->k, ii = st->ii;
    const int l = j_local;
    if (l < k || l == ii) return;
    const double2 d = jdot_block(A + (size_t)ii * lda, A + (size_t)l * lda, J, k, m, red);
    if (threadIdx.x == 0) hi[l] = sqrt(cnorm2(d));
}

// Second Bunch-Kaufman test, the swaps it implies, and for a 2x2 pivot the
// Jacobi rotation of the pivot J-Gram applied to columns k, k+1.
__global__ __launch_bounds__(kOneNT) void k_jqr_decide2(const PencilDev *PD) {
    __shared__ double red[4 * kOneNT / kWave];
    __shared__ double rv[kOneNT / kWave];
    __shared__ int ri[kOneNT / kWave];
    __shared__ int piv_s, swp_s;
    JQR_PENCIL_ONE();
    double *hd = P.hd;
    const double *hi = P.hi;
    int *perm = P.perm;
    if (!jqr_active(st, n) || !st->need2) return;
    const int k = st->k, ii = st->ii;
    double sv = -1.0;
    int si = k;
    for (int l = k + threadIdx.x; l < n; l += blockDim.x) {
        if (l == ii) continue;
        const double v = hi[l];
        if (v > sv || (v == sv && l < si)) { sv = v; si = l; }
    }
    block_argmax(sv, si, rv, ri);
    if (threadIdx.x == 0) {
        const double alpha = (1.0 + sqrt(17.0)) / 8.0;
        const double lam = st->lam;
        int piv = 1, swp = -1;
        if (fabs(hd[k]) * sv >= alpha * lam * lam) {
            piv = 1;
        } else if (fabs(hd[ii]) >= alpha * sv) {
            piv = 1;
            swp = k;
        } else {
            piv = 2;
            if (ii != k + 1) swp = k + 1;
        }
        if (swp >= 0) {
            const int t = perm[swp]; perm[swp] = perm[ii]; perm[ii] = t;
            const double h = hd[swp]; hd[swp] = hd[ii]; hd[ii] = h;
        }
        piv_s = piv;
        swp_s = swp;
        st->piv = piv;
    }
    __syncthreads();
    if (swp_s >= 0) swap_cols_block(A, lda, m, swp_s, ii);
    if (piv_s != 2) return;
    __syncthreads();
    // 2x2 pivot: J-Gram of columns k, k+1 over rows k..m-1.
    double2 *x = A + (size_t)k * lda;
    double2 *y = A + (size_t)(k + 1) * lda;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = k + threadIdx.x; r < m; r += blockDim.x) {
        const double s = jsign(J, r);
        const double2 a = x[r], b = y[r];
        v[0] += s * cnorm2(a);
        v[1] += s * cnorm2(b);
        v[2] += s * (a.x * b.x + a.y * b.y);
        v[3] += s * (a.x * b.y - a.y * b.x);
    }
    block_sum<4>(v, red);
    const double h11 = v[0], h22 = v[1];
    const double ah = sqrt(v[2] * v[2] + v[3] * v[3]);
    double co = 1.0, sn = 0.0;
    double2 e = cmk(1.0, 0.0);
    if (ah > 0.0) {
        e = cmk(v[2] / ah, v[3] / ah);
        const double tt = (h22 - h11) / (2.0 * ah);
        const double tn = (tt >= 0.0 ? 1.0 : -1.0) / (fabs(tt) + sqrt(1.0 + tt * tt));
        co = 1.0 / sqrt(1.0 + tn * tn);
        sn = tn * co;
    }
    // [x, y] <- [x, y] R, R = [[co, e sn], [-conj(e) sn, co]]
    for (int r = k + threadIdx.x; r < m; r += blockDim.x) {
        const double2 a = x[r], b = y[r];
        const double2 ecb = cmulc(e, b);  // conj(e) * b
        const double2 eb = cmul(e, a);
        x[r] = csub(cscale(a, co), cscale(ecb, sn));
        y[r] = cadd(cscale(eb, sn), cscale(b, co));
    }
    if (threadIdx.x == 0) {
        st->co = co;
        st->si = sn;
        st->eph = e;
    }
}

// Builds the hyperbolic reflector for column c = k + which, rows r0 = c..m-1.
__global__ __launch_bounds__(kOneNT) void k_jqr_reflect(const PencilDev *PD, int which) {
    __shared__ double red[kOneNT / kWave];
    __shared__ double rv[kOneNT / kWave];
    __shared__ int ri[kOneNT / kWave];
    JQR_PENCIL_ONE();
    double2 *sbuf = P.sbuf;
    if (!jqr_active(st, n)) return;
    if (which == 1 && st->piv != 2) return;
    const int c = st->k + which;
    const int r0 = c;
    double2 *x = A + (size_t)c * lda;
    const double h = jnorm_block(x, J, r0, m, red);
    if (!isfinite(h) || h == 0.0) {
        if (threadIdx.x == 0) st->status = isfinite(h) ? GHSVD_ERANK : GHSVD_ENONFINITE;
        return;
    }
    const int8_t sg = h > 0.0 ? 1 : -1;
    if (J[r0] != sg) {
        // the matching-sign row with the largest |f_i| comes to the front
        double bv = -1.0;
        int bi = -1;
        for (int r = r0 + threadIdx.x; r < m; r += blockDim.x) {
            if (J[r] == sg) {
                const double v = cnorm2(x[r]);
                if (v > bv || (v == bv && (bi < 0 || r < bi))) { bv = v; bi = r; }
            }
        }
        if (bi < 0) bi = 0x7fffffff;
        block_argmax(bv, bi, rv, ri);
        if (bi < r0 || bi >= m) {
            if (threadIdx.x == 0) st->status = GHSVD_ERANK;
            return;
        }
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double2 *col = A + (size_t)j * lda;
            const double2 t = col[r0];
            col[r0] = col[bi];
            col[bi] = t;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            J[bi] = J[r0];
            J[r0] = sg;
        }
    }
    __syncthreads();
    const double2 f11 = x[r0];
    __syncthreads();  // every wavefront has read f_11 before it is overwritten
    const double af = sqrt(cnorm2(f11));
    const double2 e = af > 0.0 ? cmk(f11.x / af, f11.y / af) : cmk(1.0, 0.0);
    const double rr = sqrt(fabs(h));
    double2 *s = sbuf + (size_t)which * m;
    for (int r = r0 + 1 + threadIdx.x; r < m; r += blockDim.x) {
        s[r] = x[r];
        x[r] = cmk(0.0, 0.0);
    }
    if (threadIdx.x == 0) {
        s[r0] = cscale(e, af + rr);
        x[r0] = cscale(e, -rr);  // -c_1
        st->tau[which] = -1.0 / (h + rr * af * (double)sg);
    }
}

// Applies H(s) = I + tau s s^* J to columns j > c (rows r0..m-1) and, when
// the next iteration starts after this reflector, leaves the columns'
// J-norms over rows c+1..m-1 in hd.
__global__ __launch_bounds__(kGridNT) void k_jqr_apply(const PencilDev *PD, const int *pre, int B,
                                                       int which) {
    __shared__ double red[2 * kGridNT / kWave];
    JQR_PENCIL_COL();
    const double2 *sbuf = P.sbuf;
    double *hd = P.hd;
    if (!jqr_active(st, n)) return;
    const int piv = st->piv;
    if (which == 1 && piv != 2) return;
    const int c = st->k + which;
    const int r0 = c;
    const int j = j_local;
    if (j <= c) return;
    const double2 *s = sbuf + (size_t)which * m;
    double2 *y = A + (size_t)j * lda;
    const double2 w = jdot_block(s, y, J, r0, m, red);
    const double2 tw = cscale(w, st->tau[which]);
    const bool last = (which == 1) || (piv == 1);
    double v[1] = {0.0};
    for (int r = r0 + threadIdx.x; r < m; r += blockDim.x) {
        const double2 nv = cadd(y[r], cmul(s[r], tw));
        y[r] = nv;
        if (r > r0) v[0] += jsign(J, r) * cnorm2(nv);
    }
    if (last) {
        block_sum<1>(v, red);
        if (threadIdx.x == 0) hd[j] = v[0];
    }
}

// Finishes a 2x2 pivot (R^* on rows k, k+1 of the pivot block) and advances k.
__global__ void k_jqr_finish(const PencilDev *PD) {
    JQR_PENCIL_ONE();
    if (!jqr_active(st, n)) return;
    if (threadIdx.x != 0) return;
    const int k = st->k;
    if (st->piv == 2) {
        const double co = st->co, sn = st->si;
        const double2 e = st->eph;
        double2 *x = A + (size_t)k * lda;
        double2 *y = A + (size_t)(k + 1) * lda;
        for (int r = k; r < k + 2; ++r) {
            const double2 a = x[r], b = y[r];
            // [x, y] <- [x, y] R^*, R^* = [[co, -e sn], [conj(e) sn, co]]
            x[r] = cadd(cscale(a, co), cscale(cmulc(e, b), sn));
            y[r] = csub(cscale(b, co), cscale(cmul(e, a), sn));
        }
        st->n2x2 += 1;
    }
    st->k = k + st->piv;
}

__global__ void k_jqr_init(const PencilDev *PD) {
    const PencilDev P = PD[blockIdx.x];
    JqrState *st = P.jst;
    int *perm = P.perm;
    const int n = P.n;
    const int t = threadIdx.x;
    for (int j = t; j < n; j += blockDim.x) perm[j] = j;
    if (!P.reduce) return;
    if (t == 0) {
        st->k = 0;
        st->piv = 1;
        st->need2 = 0;
        st->ii = 0;
        st->status = 0;
        st->n2x2 = 0;
    }
}

// ---------------------------------------------------------------------------
// Householder QR of G P2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kOneNT) void k_qr_house(const PencilDev *PD, int k) {
    __shared__ double red[kOneNT / kWave];
    const PencilDev P = PD[blockIdx.x];
    if (!P.reduce || k >= P.n || P.jst->status != 0) return;
    double2 *A = P.Gt;
    const long lda = P.ldgt;
    const int p = P.p;
    double2 *v = P.qv;
    double *coef = P.qcoef;
    double2 *x = A + (size_t)k * lda;
    double s[1] = {0.0};
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) s[0] += cnorm2(x[r]);
    block_sum<1>(s, red);
    const double nrm = sqrt(s[0]);
    if (nrm == 0.0) {
        if (threadIdx.x == 0) coef[0] = 0.0;
        return;
    }
    const double2 x1 = x[k];
    __syncthreads();  // every wavefront has read x_1 before it is overwritten
    const double ax1 = sqrt(cnorm2(x1));
    const double2 ph = ax1 > 0.0 ? cmk(x1.x / ax1, x1.y / ax1) : cmk(1.0, 0.0);
    for (int r = k + 1 + threadIdx.x; r < p; r += blockDim.x) {
        v[r] = x[r];
        x[r] = cmk(0.0, 0.0);
    }
    if (threadIdx.x == 0) {
        v[k] = cscale(ph, ax1 + nrm);
        x[k] = cscale(ph, -nrm);
        coef[0] = 1.0 / (nrm * (nrm + ax1));  // 2 / (v^* v)
    }
}

__global__ __launch_bounds__(kGridNT) void k_qr_apply(const PencilDev *PD, const int *pre, int B,
                                                      int k) {
    __shared__ double red[2 * kGridNT / kWave];
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev P = PD[pk];
    if (!P.reduce || k >= P.n || P.jst->status != 0) return;
    const int j = blockIdx.x - pre[pk];
    if (j <= k) return;
    double2 *A = P.Gt;
    const long lda = P.ldgt;
    const int p = P.p;
    const double2 *v = P.qv;
    const double cf = P.qcoef[0];
    if (cf == 0.0) return;
    double2 *y = A + (size_t)j * lda;
    double w[2] = {0.0, 0.0};
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) {
        const double2 a = v[r], b = y[r];
        w[0] += a.x * b.x + a.y * b.y;
        w[1] += a.x * b.y - a.y * b.x;
    }
    block_sum<2>(w, red);
    const double2 tw = cmk(w[0] * cf, w[1] * cf);
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) y[r] = csub(y[r], cmul(v[r], tw));
}

// ---------------------------------------------------------------------------
// Copies, signature split, input checks.
// ---------------------------------------------------------------------------
__global__ void k_copy_cols(int rows, const double2 *src, long lds, double2 *dst, long ldd,
                            const int *perm) {
    const int j = blockIdx.y;
    const int sj = perm ? perm[j] : j;
    const double2 *s = src + (size_t)sj * lds;
    double2 *d = dst + (size_t)j * ldd;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        d[r] = s[r];
}

int copy_cols(int rows, int n, const double2 *src, long lds, double2 *dst, long ldd,
              const int *perm, hipStream_t stream) {
    int bx = (rows + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_copy_cols, dim3(bx, n), dim3(256), 0, stream, rows, src, lds, dst, ldd,
                       perm);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// rowmap[r] = destination row of source row r (stable: + rows keep their
// order at the front, - rows keep theirs after them).
__global__ __launch_bounds__(kOneNT) void k_jsplit_map(int rows, const int8_t *J, int *rowmap,
                                                       int *nplus) {
    __shared__ int warp_tot[kOneNT / kWave];
    __shared__ int base_s;
    __shared__ int total_plus;
    const int lane = threadIdx.x & 63, wid = threadIdx.x / 64, nw = blockDim.x / 64;
    // pass 1: count + rows
    int cnt = 0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) cnt += (J[r] > 0);
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0) warp_tot[wid] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < nw; ++w) t += warp_tot[w];
        total_plus = t;
        base_s = 0;
        nplus[0] = t;
    }
    __syncthreads();
    const int np = total_plus;
    // pass 2: chunked exclusive scan of the + flags
    for (int c0 = 0; c0 < rows; c0 += blockDim.x) {
        const int r = c0 + threadIdx.x;
        const int f = (r < rows && J[r] > 0) ? 1 : 0;
        // inclusive scan within the wavefront
        int incl = f;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        if (lane == 63) warp_tot[wid] = incl;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < wid; ++w) wbase += warp_tot[w];
        const int before = base_s + wbase + incl - f;  // + rows before r
        if (r < rows) rowmap[r] = f ? before : np + (r - before);
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) base_s += wbase + incl;
        __syncthreads();
    }
}

__global__ void k_jsplit_copy(int rows, const double2 *src, long lds, double2 *dst, long ldd,
                              const int *rowmap) {
    const int j = blockIdx.y;
    const double2 *s = src + (size_t)j * lds;
    double2 *d = dst + (size_t)j * ldd;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        d[rowmap[r]] = s[r];
}

int jsplit(int rows, int n, const double2 *src, long lds, const int8_t *J, double2 *dst, long ldd,
           int *rowmap, int *nplus_dev, hipStream_t stream) {
    hipLaunchKernelGGL(k_jsplit_map, dim3(1), dim3(kOneNT), 0, stream, rows, J, rowmap, nplus_dev);
    int bx = (rows + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_jsplit_copy, dim3(bx, n), dim3(256), 0, stream, rows, src, lds, dst, ldd,
                       rowmap);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

__global__ void k_check(int m, int n, int p, const double2 *F, long ldf, const int8_t *J,
                        const double2 *G, long ldg, int *flags, double *gnorm2) {
    __shared__ double red[256 / kWave];
    const int j = blockIdx.y;
    int bad = 0;
    double g2[1] = {0.0};
    if (j == 0) {
        for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < m; r += gridDim.x * blockDim.x)
            if (J[r] != 1 && J[r] != -1) bad |= 1;
    }
    const double2 *f = F + (size_t)j * ldf;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < m; r += gridDim.x * blockDim.x) {
        const double2 a = f[r];
        if (!isfinite(a.x) || !isfinite(a.y)) bad |= 2;
    }
    const double2 *g = G + (size_t)j * ldg;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < p; r += gridDim.x * blockDim.x) {
        const double2 a = g[r];
        if (!isfinite(a.x) || !isfinite(a.y)) bad |= 2;
        g2[0] += cnorm2(a);
    }
    if (bad) atomicOr(flags, bad);
    block_sum<1>(g2, red);
    if (threadIdx.x == 0) atomicAdd(gnorm2, g2[0]);
}

int check_inputs(int m, int n, int p, const double2 *F, long ldf, const int8_t *J,
                 const double2 *G, long ldg, int *flags, double *gnorm2, hipStream_t stream) {
    int rows = m > p ? m : p;
    int bx = (rows + 255) / 256;
    if (bx > 8) bx = 8;
    hipLaunchKernelGGL(k_check, dim3(bx, n), dim3(256), 0, stream, m, n, p, F, ldf, J, G, ldg,
                       flags, gnorm2);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

__global__ void k_identity(int n, void *Z, long ldz, int fp32) {
    const int j = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const double v = (r == j) ? 1.0 : 0.0;
        if (fp32)
            reinterpret_cast<float2 *>(Z)[(size_t)j * ldz + r] = make_float2((float)v, 0.0f);
        else
            reinterpret_cast<double2 *>(Z)[(size_t)j * ldz + r] = make_double2(v, 0.0);
    }
}

int set_identity(int n, void *Z, long ldz, int fp32, hipStream_t stream) {
    int bx = (n + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_identity, dim3(bx, n), dim3(256), 0, stream, n, Z, ldz, fp32);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

__global__ void k_jqr_status(const PencilDev *PD, int B, int *out) {
    for (int k = threadIdx.x; k < B; k += blockDim.x) {
        const PencilDev P = PD[k];
        if (!P.reduce) {
            out[2 * k] = 0;
            out[2 * k + 1] = 0;
            continue;
        }
        const JqrState *st = P.jst;
        out[2 * k] = st->status ? st->status : (st->k < P.n ? GHSVD_ERANK : 0);
        out[2 * k + 1] = st->n2x2;
    }
}

int run_reduction(const BatchCtx &c, std::vector<int> &status, std::vector<int> &n2x2,
                  hipStream_t s) {
    const int B = c.B;
    status.assign(B, 0);
    n2x2.assign(B, 0);
    int any = 0;
    for (const PencilDev &P : c.host) any |= P.reduce;
    if (!any) return GHSVD_OK;
    for (int k = 0; k < B; ++k) {
        const PencilDev &P = c.host[k];
        if (!P.reduce) continue;
        int rc = copy_cols(P.m, P.n, P.Fin, P.ldfin, P.Ft, P.ldft, nullptr, s);
        if (rc) return rc;
        GHSVD_HIP(hipMemcpyAsync(P.Jw, P.Jin, (size_t)P.m, hipMemcpyDeviceToDevice, s));
    }
    const int *pc = c.pre_of(BatchCtx::kCols);
    const int tot = c.total(BatchCtx::kCols);
    hipLaunchKernelGGL(k_jqr_init, dim3(B), dim3(256), 0, s, c.dev);
    hipLaunchKernelGGL(k_jqr_colnorms, dim3(tot), dim3(kGridNT), 0, s, c.dev, pc, B);
    // At most max_n iterations (fewer when 2x2 pivots occur; extra ones exit at once).
    for (int it = 0; it < c.max_n; ++it) {
        hipLaunchKernelGGL(k_jqr_cross, dim3(tot), dim3(kGridNT), 0, s, c.dev, pc, B);
        hipLaunchKernelGGL(k_jqr_decide1, dim3(B), dim3(kOneNT), 0, s, c.dev);
        hipLaunchKernelGGL(k_jqr_cross2, dim3(tot), dim3(kGridNT), 0, s, c.dev, pc, B);
        hipLaunchKernelGGL(k_jqr_decide2, dim3(B), dim3(kOneNT), 0, s, c.dev);
        for (int w = 0; w < 2; ++w) {
            hipLaunchKernelGGL(k_jqr_reflect, dim3(B), dim3(kOneNT), 0, s, c.dev, w);
            hipLaunchKernelGGL(k_jqr_apply, dim3(tot), dim3(kGridNT), 0, s, c.dev, pc, B, w);
        }
        hipLaunchKernelGGL(k_jqr_finish, dim3(B), dim3(64), 0, s, c.dev);
    }
    GHSVD_HIP(hipGetLastError());
    for (int k = 0; k < B; ++k) {
        const PencilDev &P = c.host[k];
        if (!P.reduce) continue;
        int rc = copy_cols(P.p, P.n, P.Gin, P.ldgin, P.Gt, P.ldgt, P.perm, s);
        if (rc) return rc;
    }
    for (int k = 0; k < c.max_n; ++k) {
        hipLaunchKernelGGL(k_qr_house, dim3(B), dim3(kOneNT), 0, s, c.dev, k);
        hipLaunchKernelGGL(k_qr_apply, dim3(tot), dim3(kGridNT), 0, s, c.dev, pc, B, k);
    }
    GHSVD_HIP(hipGetLastError());
    std::vector<int> out(2 * B);
    hipLaunchKernelGGL(k_jqr_status, dim3(1), dim3(256), 0, s, c.dev, B, c.done_dev);
    GHSVD_HIP(hipMemcpyAsync(out.data(), c.done_dev, sizeof(int) * 2 * B, hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < B; ++k) {
        status[k] = out[2 * k];
        n2x2[k] = out[2 * k + 1];
    }
    return GHSVD_OK;
}

}  // namespace ghsvd
