// reduce.hip -- one-time reduction of tall F, G to square factors (Section 5).
//
// F: hyperbolic QR (JQR, eq. (5.1)) with diagonal pivoting supplemented by
// Bunch-Kaufman partial pivoting (Section 5.2.1, alpha = (1 + sqrt(17)) / 8),
// single pivots reduced by the hyperbolic Householder reflector H(s) of
// Section 5.3 (Theorem 5.1, generator s = f + c_1 e_1 with arg c_1 = arg f_11,
// a matching-sign row swapped to the front when needed), 2x2 pivots by the
// (J, I) URV step (Jacobi rotation of the pivot J-Gram, two reflectors, R^*).
// G: Householder QR of G without pivoting (Q is not formed); the caller
// permutes the triangular factor's columns by P2.  The iteration sees G only
// through G^*G, and R_G P2 has the Gram of the triangular factor of G P2, so
// the QR needs no pivot decision: its column steps ride in the hyperbolic
// QR's step launches as extra workgroups.
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
// Trailing columns per workgroup of the step kernel where F's columns fit the
// register-resident step at up to 6 rows per thread (the pivot's reflector is
// formed once for all of them); other windows keep one column per workgroup.
constexpr int kStepCols = 2;
// Blocked QR of G: panel width, the longest column the trailing kernel
// holds in registers, columns per trailing workgroup.
constexpr int kQrPanel = 32;
constexpr int kQrRegRows = 2048;
constexpr int kQrTrailCols = 4;

__device__ __forceinline__ double jsign(const int8_t *J, int r) { return (double)J[r]; }

// Complex products with the FMA contraction spelled out: the register-
// resident step forms below use these so that they round exactly as the
// compiled streaming loops of the same step do (which product of a sum is
// fused is otherwise the compiler's choice, and it differs between the two
// forms).  fnorm2, fdot_*, fmul: the first product fused, the second rounded;
// fdot_re2: the second fused (the streaming reflector J-product's form).
__device__ __forceinline__ double fnorm2(double2 a) { return __builtin_fma(a.x, a.x, a.y * a.y); }
// conj(a) * b, real and imaginary parts
__device__ __forceinline__ double fdot_re(double2 a, double2 b) {
    return __builtin_fma(a.x, b.x, a.y * b.y);
}
__device__ __forceinline__ double fdot_re2(double2 a, double2 b) {
    return __builtin_fma(a.y, b.y, a.x * b.x);
}
__device__ __forceinline__ double fdot_im(double2 a, double2 b) {
    return __builtin_fma(a.x, b.y, -(a.y * b.x));
}
// a * b
__device__ __forceinline__ double2 fmul(double2 a, double2 b) {
    return cmk(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}

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

__device__ __forceinline__ bool jqr_active(const JqrState &st, int n) {
    return st.status == 0 && st.k < n;
}

// Batched launches over columns: workgroup -> (pencil, logical column j)
// through prefix sums of column counts.  A launch of step `it` covers only the
// columns j >= jw of each pencil, jw = it rounded down to the window step
// (k >= it for a pencil still in its factorization, so no live column lies
// left of the window); the prefix sums of the window's column counts come
// from a host-built table with one row per window.  Columns never move: logical
// column l of the factorization is physical column perm[l] of Ft (the map
// is P2), and a step's two swaps only change the map.  State, signature and
// map are read from the copies of the step's parity `par`.
#define JQR_PENCIL_COL() JQR_PENCIL_COL_AT((int)blockIdx.x)
#define JQR_PENCIL_COL_AT(BLK)                                    \
    const int blk_ = (BLK);                                       \
    const int pk = find_pencil(pre, B, blk_);                     \
    const PencilDev P = PD[pk];                                  \
    if (!P.reduce) return;                                        \
    const double2 *A = P.Ft;                                      \
    const long lda = P.ldft;                                      \
    const int m = P.m, n = P.n;                                   \
    const JqrState st = P.jst[par];                               \
    const int8_t *J = P.Jw + (size_t)par * m;                     \
    const int j_local = pencil_local(pre, pk, blk_) + jw;         \
    (void)J;                                                      \
    (void)j_local

__device__ __forceinline__ const double2 *jcol(const double2 *A, long lda, int c) {
    return A + (size_t)c * lda;
}

// Diagonal pivot of step k: the logical column i >= k with the largest
// |J-norm^2| (the first one on ties), the same in every workgroup.  hl holds
// the J-norms by logical column, so no column map is read first.
__device__ __forceinline__ int jqr_diag_pivot(const double *hl, int k, int n, double *rv, int *ri) {
    double bv = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(hl[i]);
        if (v > bv || (v == bv && i < bi)) {
            bv = v;
            bi = i;
        }
    }
    block_argmax(bv, bi, rv, ri);
    return bi;
}

// hd[c] = J-norm^2 of every column over rows 0..m-1 (before the first step),
// and hl[j] for its logical column j.
__global__ __launch_bounds__(kGridNT) void k_jqr_colnorms(const PencilDev *PD, const int *pre, int B,
                                                          int par, int jw) {
    __shared__ double red[kGridNT / kWave];
    JQR_PENCIL_COL();
    if (!jqr_active(st, n)) return;
    const int c = P.perm[j_local];
    const double h = jnorm_block(jcol(A, lda, c), J, st.k, m, red);
    if (threadIdx.x == 0) {
        P.hd[c] = h;
        P.hl[j_local] = h;
    }
}

// Step, first kernel: every workgroup finds the diagonal pivot bi, and the
// workgroup of logical column j computes the J-product of column bi with
// column j (rows k..m-1), stored at the position column j takes after the
// swap k <-> bi.  Workgroups take the columns in the reverse of the step
// kernel's order: workgroups start roughly in index order, so the columns the
// previous step kernel wrote last, the ones most likely still held in the
// memory-side cache, are read first (and the next step kernel starts on the
// columns this kernel read last).
__global__ __launch_bounds__(kGridNT) void k_jqr_cross(const PencilDev *PD, const int *pre, int B,
                                                       int par, int jw) {
    __shared__ double red[2 * kGridNT / kWave];
    __shared__ double rv[kGridNT / kWave];
    __shared__ int ri[kGridNT / kWave];
    JQR_PENCIL_COL_AT((int)(gridDim.x - 1 - blockIdx.x));
    if (!jqr_active(st, n)) return;
    const int k = st.k, j = j_local;
    if (j < k || k == n - 1) return;
    const int *cp = P.perm;
    const int bi = jqr_diag_pivot(P.hl, k, n, rv, ri);
    if (j == k && threadIdx.x == 0) P.jdec->bi = bi;  // for the second kernel
    if (j == bi) return;
    const double2 d = jdot_block(jcol(A, lda, cp[bi]), jcol(A, lda, cp[j]), J, k, m, red);
    const int pos = (j == k) ? bi : j;
    if (threadIdx.x == 0) P.hc[pos] = d;
}

// Step, second kernel: every workgroup takes the diagonal pivot swap and the
// first Bunch-Kaufman test (Section 5.2.1, alpha = (1 + sqrt(17)) / 8) from
// the first kernel's results; the workgroup of column k records them.  When
// the second test is needed, workgroup l computes |J-product| of the
// candidate column ii with column l (post-swap positions).
__global__ __launch_bounds__(kGridNT) void k_jqr_cross2(const PencilDev *PD, const int *pre, int B,
                                                        int par, int jw) {
    __shared__ double red[2 * kGridNT / kWave];
    __shared__ double rv[kGridNT / kWave];
    __shared__ int ri[kGridNT / kWave];
    JQR_PENCIL_COL();
    if (!jqr_active(st, n)) return;
    const int k = st.k, j = j_local;
    if (j < k) return;
    const int *cp = P.perm;
    // the diagonal pivot, recorded by the first kernel (none at the last column)
    const int bi = k == n - 1 ? k : P.jdec->bi;
    // candidate ii = argmax_{i > k} |h_ki| (hc holds post-swap positions)
    double cv = -1.0;
    int ci = k + 1;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
        const double v = sqrt(cnorm2(P.hc[i]));
        if (v > cv || (v == cv && i < ci)) {
            cv = v;
            ci = i;
        }
    }
    block_argmax(cv, ci, rv, ri);
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    // |J-norm^2| of the column at position k after the swap: hl[bi] = hd[cp[bi]]
    const int need2 = (k < n - 1) && !(fabs(P.hl[bi]) >= alpha * cv);
    auto cp1 = [&](int l) { return l == k ? cp[bi] : (l == bi ? cp[k] : cp[l]); };
    if (j == k) {
        for (int l = threadIdx.x; l < n; l += blockDim.x) P.cpb[l] = cp1(l);
        if (threadIdx.x == 0) {
            JqrDecision d;
            d.bi = bi;
            d.ii = ci;
            d.need2 = need2;
            d.pad = 0;
            d.lam = cv;
            *P.jdec = d;
        }
    }
    if (!need2 || j == ci) return;
    const double2 d = jdot_block(jcol(A, lda, cp1(ci)), jcol(A, lda, cp1(j)), J, k, m, red);
    if (threadIdx.x == 0) P.hi[j] = sqrt(cnorm2(d));
}

// A column read through the row swaps of the step: rows a0 <-> b0, then
// a1 <-> b1 (either may be the identity).  Rows named by a swap are staged
// in LDS before the column is rewritten in place (sv[0..3] = rows a0, b0,
// a1, b1 of the column as stored).
struct SwapView {
    int a0, b0, a1, b1;
    __device__ int src(int r) const {
        // the row whose stored value lands at r after both swaps
        int q = r;
        if (q == a1) q = b1;
        else if (q == b1) q = a1;
        if (q == a0) q = b0;
        else if (q == b0) q = a0;
        return q;
    }
    __device__ int src0(int r) const {
        if (r == a0) return b0;
        if (r == b0) return a0;
        return r;
    }
};

__device__ __forceinline__ double2 sv_load(const double2 *x, const double2 *stash, const SwapView &v,
                                           int q) {
    if (q == v.a0) return stash[0];
    if (q == v.b0) return stash[1];
    if (q == v.a1) return stash[2];
    if (q == v.b1) return stash[3];
    return x[q];
}

// Step, third kernel.  Every workgroup takes the second Bunch-Kaufman test,
// the pivot (1x1: the hyperbolic reflector of the pivot column, Theorem 5.1,
// with a matching-sign row swapped to the front when needed; 2x2: the
// Jacobi rotation of the pivot J-Gram, one reflector per pivot column and
// R^* on the pivot rows), all from the pivot columns as stored; then the
// workgroup of each trailing column applies the reflector(s) to its column
// in place and leaves its J-norm^2 over the rows still to reduce in hd.
// The workgroup of column k writes the next state, map and signature, and
// the pivot rows; the pivot columns themselves are not rewritten (the final
// extraction takes their rows from rblk and zeros below them).  A final
// state (factorization complete, or an error) goes to both parity copies, so
// the later steps, which have no workgroup for a finished pencil, need not
// carry it.
template <int RC>
__device__ __forceinline__ void qr_step_body(const PencilDev *PD, const int *pre, int B, int k,
                                             int bid, int jw, double *red);
template <int RC>
__device__ __forceinline__ void qr_panel_body(const PencilDev *PD, int B, int k, int bid,
                                              double *red);

// A 1x1 pivot step with the workgroup's rows in registers: thread tid holds
// rows k + tid + i * kGridNT (i < RC) of the signature, the pivot column and
// the workgroup's own columns j0, j0 + 1, ... (those right of k), loaded
// together at the start (one memory latency), which is the row assignment of
// the streaming loops below, so every sum rounds as there.  The pivot's
// J-norm, row search and reflector are formed once for all the workgroup's
// columns, and their J-products and J-norms share each workgroup reduction
// (every component is summed in the same order as alone).  The row swap
// k <-> b0 of the matching sign moves the values between the two owning
// threads through LDS.  Requires m - k <= RC * kGridNT.
template <int RC, int NC, typename CP>
__device__ __forceinline__ void jqr_step1_regs(const PencilDev &P, const JqrState &cur, int par,
                                               int k, int j0, const CP &cp2, double *red,
                                               double *rv, int *ri, double2 *xch) {
    const int m = P.m, n = P.n, tid = threadIdx.x;
    bool tr[NC];  // column j0 + c is a trailing column of this step
    bool desig = false, any = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int j = j0 + c;
        tr[c] = j > k && j < n;
        desig |= j == k;
        any |= tr[c];
    }
    int8_t *Jc = P.Jw + (size_t)par * m;
    int8_t *Jn = P.Jw + (size_t)(par ^ 1) * m;
    const double2 *xa = jcol(P.Ft, P.ldft, cp2(k));
    double2 *y[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = tr[c] ? P.Ft + (size_t)cp2(j0 + c) * P.ldft : P.Ft;
    const int jk = Jc[k];
    const double2 xk = xa[k];
    double2 xv[RC], yv[NC][RC];
    int js[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        const int r = k + tid + i * kGridNT;
        js[i] = 0;
        xv[i] = cmk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NC; ++c) yv[c][i] = cmk(0.0, 0.0);
        if (r < m) {
            js[i] = Jc[r];
            xv[i] = xa[r];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (tr[c]) yv[c][i] = y[c][r];
        }
    }
    int status = 0;
    double h0;
    {
        double v[1] = {0.0};
#pragma unroll
        for (int i = 0; i < RC; ++i)
            if (k + tid + i * kGridNT < m) v[0] += (double)js[i] * fnorm2(xv[i]);
        block_sum<1>(v, red);
        h0 = v[0];
    }
    if (!isfinite(h0) || h0 == 0.0) status = isfinite(h0) ? GHSVD_ERANK : GHSVD_ENONFINITE;
    const int sg0 = h0 > 0.0 ? 1 : -1;
    int b0 = k;
    if (status == 0 && jk != sg0) {
        double bv = -1.0;
        int bi = -1;
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = k + tid + i * kGridNT;
            if (r < m && js[i] == sg0) {
                const double v = fnorm2(xv[i]);
                if (v > bv || (v == bv && (bi < 0 || r < bi))) {
                    bv = v;
                    bi = r;
                }
            }
        }
        if (bi < 0) bi = 0x7fffffff;
        block_argmax(bv, bi, rv, ri);
        if (bi < k || bi >= m) status = GHSVD_ERANK;
        else b0 = bi;
    }
    if (status != 0) {
        // every workgroup of the pencil reaches this branch (same pivot data)
        if (desig) {
            for (int r = tid; r < m; r += blockDim.x) Jn[r] = Jc[r];
            if (tid == 0) {
                JqrState t = cur;
                t.status = status;
                P.jst[par ^ 1] = t;
                P.jst[par] = t;
            }
        }
        return;
    }
    double2 f11 = xk;
    if (b0 != k) {
        // rows k and b0 trade places: J, the pivot column (as the reflector
        // sees it) and the own columns (xch: the pivot's and the columns'
        // rows b0, then the columns' rows k)
        const int ow = (b0 - k) & (kGridNT - 1);
        if (tid == ow) {
#pragma unroll
            for (int i = 0; i < RC; ++i)
                if (k + tid + i * kGridNT == b0) {
                    xch[0] = xv[i];
#pragma unroll
                    for (int c = 0; c < NC; ++c) xch[1 + c] = yv[c][i];
                }
        }
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) xch[1 + NC + c] = yv[c][0];
        }
        __syncthreads();
        f11 = xch[0];
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) yv[c][0] = xch[1 + c];
            js[0] = sg0;
        }
        if (tid == ow) {
#pragma unroll
            for (int i = 0; i < RC; ++i)
                if (k + tid + i * kGridNT == b0) {
                    xv[i] = xk;
#pragma unroll
                    for (int c = 0; c < NC; ++c) yv[c][i] = xch[1 + NC + c];
                    js[i] = jk;
                }
        }
    }
    const double af = sqrt(fnorm2(f11));
    const double2 e = af > 0.0 ? cmk(f11.x / af, f11.y / af) : cmk(1.0, 0.0);
    const double rr = sqrt(fabs(h0));
    const double2 s0k = cscale(e, af + rr);
    const double2 r0k = cscale(e, -rr);
    const double tau0 = -1.0 / (h0 + rr * af * (double)sg0);
    if (desig) {
        const bool fin = k + 1 >= n;
        for (int l = tid; l < n; l += blockDim.x) P.perm[l] = cp2(l);
        for (int r = tid; r < k; r += blockDim.x) Jn[r] = Jc[r];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = k + tid + i * kGridNT;
            if (r < m) {
                Jn[r] = (int8_t)js[i];
                if (fin) Jc[r] = (int8_t)js[i];
            }
        }
        if (tid == 0) {
            P.rblk[2 * k] = r0k;
            P.rblk[2 * k + 1] = cmk(0.0, 0.0);
            P.pblk[2 * k] = k;
            P.pblk[2 * k + 1] = 1;
            JqrState t = cur;
            t.k = k + 1;
            P.jst[par ^ 1] = t;
            if (fin) P.jst[par] = t;
        }
    }
    if (!any) return;
    // the reflector on the own columns: the J-products, then the update and
    // each column's J-norm^2 over the rows still to reduce
    double v[2 * NC];
#pragma unroll
    for (int q = 0; q < 2 * NC; ++q) v[q] = 0.0;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        const int r = k + tid + i * kGridNT;
        if (r < m) {
            const double s = (double)js[i];
            const double2 a = r == k ? s0k : xv[i];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                v[2 * c] += s * fdot_re2(a, yv[c][i]);
                v[2 * c + 1] += s * fdot_im(a, yv[c][i]);
            }
        }
    }
    block_sum<2 * NC>(v, red);
    double2 tw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) tw[c] = cscale(cmk(v[2 * c], v[2 * c + 1]), tau0);
    double h[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) h[c] = 0.0;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        const int r = k + tid + i * kGridNT;
        if (r < m) {
            const double2 a = r == k ? s0k : xv[i];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (tr[c]) {
                    const double2 nv = cadd(yv[c][i], fmul(a, tw[c]));
                    if (r > k) h[c] += (double)js[i] * fnorm2(nv);
                    y[c][r] = nv;
                }
        }
    }
    block_sum<NC>(h, red);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (tr[c]) {
                P.hd[cp2(j0 + c)] = h[c];
                P.hl[j0 + c] = h[c];
            }
    }
}

// Workgroup g < tot of the launch takes the window's columns jw + NC g' ..
// + NC - 1 of its pencil (g' its index within the pencil, from the prefix
// sums pre2 of the pencils' groups of NC columns); workgroups tot.. run
// column step qk of G's QR instead (pre: the prefix sums of columns).  RC,
// RCG: rows per thread of the register-resident 1x1 step of F and of G's
// column step; longer columns, and 2x2 pivots, take the streaming loops.
template <int RC, int RCG, int NC>
__global__ __launch_bounds__(kGridNT) void k_jqr_step(const PencilDev *PD, const int *pre,
                                                      const int *pre2, int B, int par, int tot,
                                                      int qk, int jw, int qpanel) {
    extern __shared__ int8_t Jl[];  // signature with this step's row swaps
    __shared__ double red[4 * kGridNT / kWave];
    __shared__ double rv[kGridNT / kWave];
    __shared__ int ri[kGridNT / kWave];
    __shared__ double2 stash[2 + 2 * NC];
    if ((int)blockIdx.x >= tot) {
        if (qpanel)
            qr_panel_body<RCG>(PD, B, qk, (int)blockIdx.x - tot, red);
        else
            qr_step_body<RCG>(PD, pre, B, qk, (int)blockIdx.x - tot, jw, red);
        return;
    }
    const int pk = find_pencil(pre2, B, blockIdx.x);
    const PencilDev P = PD[pk];
    if (!P.reduce) return;
    double2 *A = P.Ft;
    const long lda = P.ldft;
    const int m = P.m, n = P.n;
    const JqrState cur = P.jst[par];
    JqrState *nxt = P.jst + (par ^ 1);
    int8_t *Jc = P.Jw + (size_t)par * m;
    int8_t *Jn = P.Jw + (size_t)(par ^ 1) * m;
    const int j0 = NC * pencil_local(pre2, pk, blockIdx.x) + jw;
    const int tid = threadIdx.x;
    if (!jqr_active(cur, n)) return;
    const int k = cur.k;
    if (j0 + NC <= k) return;  // every column of the workgroup is left of k
    const bool desig = j0 <= k && k < j0 + NC;
    const JqrDecision dec = *P.jdec;
    const int *cpb = P.cpb;
    // second Bunch-Kaufman test
    int piv = 1, swp = -1;
    const int ii = dec.ii;
    if (dec.need2) {
        double sv = -1.0;
        int si = k;
        for (int l = k + tid; l < n; l += blockDim.x) {
            if (l == ii) continue;
            const double v = P.hi[l];
            if (v > sv || (v == sv && l < si)) {
                sv = v;
                si = l;
            }
        }
        block_argmax(sv, si, rv, ri);
        const double alpha = (1.0 + sqrt(17.0)) / 8.0;
        const double lam = dec.lam;
        if (fabs(P.hd[cpb[k]]) * sv >= alpha * lam * lam) {
            piv = 1;
        } else if (fabs(P.hd[cpb[ii]]) >= alpha * sv) {
            piv = 1;
            swp = k;
        } else {
            piv = 2;
            if (ii != k + 1) swp = k + 1;
        }
    }
    auto cp2 = [&](int l) {
        int q = l;
        if (swp >= 0) {
            if (l == swp) q = ii;
            else if (l == ii) q = swp;
        }
        return cpb[q];
    };
    if (piv == 1 && m - k <= RC * kGridNT) {
        jqr_step1_regs<RC, NC>(P, cur, par, k, j0, cp2, red, rv, ri, stash);
        return;
    }
    // the workgroup's columns this step rewrites: right of the pivot block
    bool any = false;
    for (int c = 0; c < NC; ++c) any |= j0 + c >= k + piv && j0 + c < n;
    if (!desig && !any) return;  // the second column of a 2x2 pivot only
    for (int r = k + tid; r < m; r += blockDim.x) Jl[r] = Jc[r];
    __syncthreads();
    const double2 *xa = jcol(A, lda, cp2(k));
    const double2 *xb = piv == 2 ? jcol(A, lda, cp2(k + 1)) : xa;
    int status = 0;
    // ---- the pivot, evaluated in every workgroup ----
    // 2x2: rotation of the pivot J-Gram over rows k..m-1
    double co = 1.0, sn = 0.0;
    double2 eph = cmk(1.0, 0.0);
    if (piv == 2) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = k + tid; r < m; r += blockDim.x) {
            const double s = (double)Jl[r];
            const double2 a = xa[r], b = xb[r];
            v[0] += s * cnorm2(a);
            v[1] += s * cnorm2(b);
            v[2] += s * (a.x * b.x + a.y * b.y);
            v[3] += s * (a.x * b.y - a.y * b.x);
        }
        block_sum<4>(v, red);
        const double h11 = v[0], h22 = v[1];
        const double ah = sqrt(v[2] * v[2] + v[3] * v[3]);
        if (ah > 0.0) {
            eph = cmk(v[2] / ah, v[3] / ah);
            const double tt = (h22 - h11) / (2.0 * ah);
            const double tn = (tt >= 0.0 ? 1.0 : -1.0) / (fabs(tt) + sqrt(1.0 + tt * tt));
            co = 1.0 / sqrt(1.0 + tn * tn);
            sn = tn * co;
        }
    }
    // rotated pivot columns at a stored row q (piv == 1: the column itself)
    auto pa = [&](int q) {
        const double2 a = xa[q];
        if (piv != 2) return a;
        const double2 b = xb[q];
        return csub(cscale(a, co), cscale(cmulc(eph, b), sn));
    };
    auto pb = [&](int q) {
        const double2 a = xa[q], b = xb[q];
        return cadd(cscale(cmul(eph, a), sn), cscale(b, co));
    };
    // reflector 0 on the first pivot column, rows k..m-1
    SwapView sw{k, k, k, k};
    double h0;
    {
        double v[1] = {0.0};
        for (int r = k + tid; r < m; r += blockDim.x) v[0] += (double)Jl[r] * cnorm2(pa(r));
        block_sum<1>(v, red);
        h0 = v[0];
    }
    if (!isfinite(h0) || h0 == 0.0) status = isfinite(h0) ? GHSVD_ERANK : GHSVD_ENONFINITE;
    int8_t sg0 = h0 > 0.0 ? 1 : -1;
    if (status == 0 && Jl[k] != sg0) {
        double bv = -1.0;
        int bi = -1;
        for (int r = k + tid; r < m; r += blockDim.x) {
            if (Jl[r] == sg0) {
                const double v = cnorm2(pa(r));
                if (v > bv || (v == bv && (bi < 0 || r < bi))) {
                    bv = v;
                    bi = r;
                }
            }
        }
        if (bi < 0) bi = 0x7fffffff;
        block_argmax(bv, bi, rv, ri);
        if (bi < k || bi >= m) status = GHSVD_ERANK;
        else sw.b0 = bi;
    }
    double2 s0k = cmk(0.0, 0.0), r0k = cmk(0.0, 0.0);
    double tau0 = 0.0;
    if (status == 0) {
        if (sw.b0 != k) {
            __syncthreads();
            if (tid == 0) {
                Jl[sw.b0] = Jl[k];
                Jl[k] = sg0;
            }
            __syncthreads();
        }
        const double2 f11 = pa(sw.b0);
        const double af = sqrt(cnorm2(f11));
        const double2 e = af > 0.0 ? cmk(f11.x / af, f11.y / af) : cmk(1.0, 0.0);
        const double rr = sqrt(fabs(h0));
        s0k = cscale(e, af + rr);
        r0k = cscale(e, -rr);
        tau0 = -1.0 / (h0 + rr * af * (double)sg0);
    }
    // s0 at row r >= k (rows of the swapped view)
    auto s0 = [&](int r) { return r == k ? s0k : pa(sw.src0(r)); };
    // 2x2: reflector 0 applied to the second pivot column, then reflector 1
    double2 w0b = cmk(0.0, 0.0), s1k = cmk(0.0, 0.0), r1k = cmk(0.0, 0.0), ybk = cmk(0.0, 0.0);
    double tau1 = 0.0;
    auto pb1 = [&](int r) {  // second pivot column after reflector 0, row r >= k
        return cadd(pb(sw.src0(r)), cmul(s0(r), cscale(w0b, tau0)));
    };
    if (piv == 2 && status == 0) {
        {
            double v[2] = {0.0, 0.0};
            for (int r = k + tid; r < m; r += blockDim.x) {
                const double s = (double)Jl[r];
                const double2 a = s0(r), b = pb(sw.src0(r));
                v[0] += s * (a.x * b.x + a.y * b.y);
                v[1] += s * (a.x * b.y - a.y * b.x);
            }
            block_sum<2>(v, red);
            w0b = cmk(v[0], v[1]);
        }
        double h1;
        {
            double v[1] = {0.0};
            for (int r = k + 1 + tid; r < m; r += blockDim.x) v[0] += (double)Jl[r] * cnorm2(pb1(r));
            block_sum<1>(v, red);
            h1 = v[0];
        }
        if (!isfinite(h1) || h1 == 0.0) status = isfinite(h1) ? GHSVD_ERANK : GHSVD_ENONFINITE;
        const int8_t sg1 = h1 > 0.0 ? 1 : -1;
        sw.a1 = sw.b1 = k + 1;
        if (status == 0 && Jl[k + 1] != sg1) {
            double bv = -1.0;
            int bi = -1;
            for (int r = k + 1 + tid; r < m; r += blockDim.x) {
                if (Jl[r] == sg1) {
                    const double v = cnorm2(pb1(r));
                    if (v > bv || (v == bv && (bi < 0 || r < bi))) {
                        bv = v;
                        bi = r;
                    }
                }
            }
            if (bi < 0) bi = 0x7fffffff;
            block_argmax(bv, bi, rv, ri);
            if (bi < k + 1 || bi >= m) status = GHSVD_ERANK;
            else sw.b1 = bi;
        }
        if (status == 0) {
            if (sw.b1 != k + 1) {
                __syncthreads();
                if (tid == 0) {
                    Jl[sw.b1] = Jl[k + 1];
                    Jl[k + 1] = sg1;
                }
                __syncthreads();
            }
            const double2 f11 = pb1(sw.b1);
            const double af = sqrt(cnorm2(f11));
            const double2 e = af > 0.0 ? cmk(f11.x / af, f11.y / af) : cmk(1.0, 0.0);
            const double rr = sqrt(fabs(h1));
            s1k = cscale(e, af + rr);
            r1k = cscale(e, -rr);
            tau1 = -1.0 / (h1 + rr * af * (double)sg1);
            ybk = pb1(k);
        }
    }
    if (status != 0) {
        // every workgroup of the pencil reaches this branch (same pivot data)
        if (desig) {
            for (int r = tid; r < m; r += blockDim.x) Jn[r] = Jc[r];
            if (tid == 0) {
                JqrState t = cur;
                t.status = status;
                *nxt = t;
                P.jst[par] = t;
            }
        }
        return;
    }
    auto s1 = [&](int r) {  // reflector 1 at row r >= k + 1
        if (r == k + 1) return s1k;
        const int q = (r == sw.b1) ? k + 1 : r;  // rows k+1 <-> b1 of the view
        return pb1(q);
    };
    if (desig) {
        // next state, map, signature, pivot rows; when the factorization ends
        // here no other workgroup of the pencil is past its early return (a
        // 2x2 pivot's second column is the last one), so the current copies
        // may be overwritten too
        const bool fin = k + piv >= n;
        for (int l = tid; l < n; l += blockDim.x) P.perm[l] = cp2(l);
        for (int r = tid; r < m; r += blockDim.x) {
            const int8_t sg = r < k ? Jc[r] : Jl[r];
            Jn[r] = sg;
            if (fin) Jc[r] = sg;
        }
        if (tid == 0) {
            if (piv == 1) {
                P.rblk[2 * k] = r0k;
                P.rblk[2 * k + 1] = cmk(0.0, 0.0);
                P.pblk[2 * k] = k;
                P.pblk[2 * k + 1] = 1;
            } else {
                // rows k, k+1 of the two pivot columns, then R^* (2x2 URV step)
                const double2 xk = r0k, xk1 = cmk(0.0, 0.0), yk = ybk, yk1 = r1k;
                const double2 a0 = xk, b0 = yk, a1 = xk1, b1 = yk1;
                P.rblk[2 * k] = cadd(cscale(a0, co), cscale(cmulc(eph, b0), sn));
                P.rblk[2 * (k + 1)] = csub(cscale(b0, co), cscale(cmul(eph, a0), sn));
                P.rblk[2 * k + 1] = cadd(cscale(a1, co), cscale(cmulc(eph, b1), sn));
                P.rblk[2 * (k + 1) + 1] = csub(cscale(b1, co), cscale(cmul(eph, a1), sn));
                P.pblk[2 * k] = k;
                P.pblk[2 * k + 1] = 2;
                P.pblk[2 * (k + 1)] = k;
                P.pblk[2 * (k + 1) + 1] = 2;
            }
            JqrState t = cur;
            t.k = k + piv;
            t.n2x2 = cur.n2x2 + (piv == 2 ? 1 : 0);
            *nxt = t;
            if (fin) P.jst[par] = t;
        }
    }
    // ---- the trailing columns: apply the reflector(s) in place ----
    for (int c = 0; c < NC; ++c) {
        const int j = j0 + c;
        if (j < k + piv || j >= n) continue;  // uniform over the workgroup
        // (the previous column's reads of the stash all precede the
        // barriers of its final reduction)
        double2 *y = A + (size_t)cp2(j) * lda;
        if (tid == 0) {
            stash[0] = y[sw.a0];
            stash[1] = y[sw.b0];
            stash[2] = y[sw.a1];
            stash[3] = y[sw.b1];
        }
        __syncthreads();
        // y0 at stored row q through the stash (rows named by a swap)
        auto y0 = [&](int q) { return sv_load(y, stash, sw, q); };
        // Jl holds both row swaps; the first reflector's dot takes J with the
        // first swap only (undo the second one, rows k+1 <-> b1)
        auto jf = [&](int r) {
            const int q = (r == sw.b1) ? sw.a1 : (r == sw.a1 ? sw.b1 : r);
            return (double)Jl[q];
        };
        double2 tw0;
        {
            double v[2] = {0.0, 0.0};
            for (int r = k + tid; r < m; r += blockDim.x) {
                const double s = jf(r);
                const double2 a = s0(r), b = y0(sw.src0(r));
                v[0] += s * (a.x * b.x + a.y * b.y);
                v[1] += s * (a.x * b.y - a.y * b.x);
            }
            block_sum<2>(v, red);
            tw0 = cscale(cmk(v[0], v[1]), tau0);
        }
        auto y1 = [&](int r) { return cadd(y0(sw.src0(r)), cmul(s0(r), tw0)); };  // r >= k
        if (piv == 1) {
            double v[1] = {0.0};
            for (int r = k + tid; r < m; r += blockDim.x) {
                const double2 nv = y1(r);
                if (r > k) v[0] += (double)Jl[r] * cnorm2(nv);
                y[r] = nv;
            }
            block_sum<1>(v, red);
            if (tid == 0) {
                P.hd[cp2(j)] = v[0];
                P.hl[j] = v[0];
            }
            continue;
        }
        double2 tw1;
        {
            double v[2] = {0.0, 0.0};
            for (int r = k + 1 + tid; r < m; r += blockDim.x) {
                const double s = (double)Jl[r];
                const int q = (r == sw.b1) ? k + 1 : (r == k + 1 ? sw.b1 : r);
                const double2 a = s1(r), b = y1(q);
                v[0] += s * (a.x * b.x + a.y * b.y);
                v[1] += s * (a.x * b.y - a.y * b.x);
            }
            block_sum<2>(v, red);
            tw1 = cscale(cmk(v[0], v[1]), tau1);
        }
        double v[1] = {0.0};
        for (int r = k + tid; r < m; r += blockDim.x) {
            double2 nv;
            if (r == k) {
                nv = y1(k);
            } else {
                const int q = (r == sw.b1) ? k + 1 : (r == k + 1 ? sw.b1 : r);
                nv = cadd(y1(q), cmul(s1(r), tw1));
                if (r > k + 1) v[0] += (double)Jl[r] * cnorm2(nv);
            }
            y[r] = nv;
        }
        block_sum<1>(v, red);
        if (tid == 0) {
            P.hd[cp2(j)] = v[0];
            P.hl[j] = v[0];
        }
    }
}

__global__ void k_jqr_init(const PencilDev *PD) {
    const PencilDev P = PD[blockIdx.x];
    int *perm = P.perm;
    const int n = P.n;
    const int t = threadIdx.x;
    for (int j = t; j < n; j += blockDim.x) perm[j] = j;
    if (!P.reduce) return;
    // until a column's pivot step records its block, the extraction reads
    // no recorded rows for it
    for (int j = t; j < n; j += blockDim.x) {
        P.pblk[2 * j] = n;
        P.pblk[2 * j + 1] = 0;
    }
    if (t == 0) {
        JqrState s;
        s.k = 0;
        s.status = 0;
        s.n2x2 = 0;
        s.pad = 0;
        P.jst[0] = s;
    }
}

// After the last step: the state and signature of the final parity move to
// the first copies (J_sq is the first n entries of Jw).
__global__ void k_jqr_settle(const PencilDev *PD, int par) {
    const PencilDev P = PD[blockIdx.x];
    if (!P.reduce || par == 0) return;
    for (int r = threadIdx.x; r < P.m; r += blockDim.x) P.Jw[r] = P.Jw[P.m + r];
    if (threadIdx.x == 0) P.jst[0] = P.jst[1];
}

// F_sq from the factored columns: logical column j, row r < n is Ft(r,
// perm[j]) above the column's pivot block, the recorded pivot rows inside
// it, and zero below; rowmap (may be NULL) moves row r to rowmap[r].
__global__ void k_jqr_extract(int n, const double2 *Ft, long ldft, const int *perm,
                              const double2 *rblk, const int *pblk, const int *rowmap,
                              double2 *dst, long ldd, int scatter) {
    const int j = blockIdx.y;
    const double2 *s = Ft + (size_t)perm[j] * ldft;
    const int kb = pblk[2 * j], bs = pblk[2 * j + 1];
    double2 *d = dst + (size_t)(scatter ? perm[j] : j) * ldd;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        double2 v;
        if (r < kb) v = s[r];
        else if (r < kb + bs) v = rblk[2 * j + (r - kb)];
        else v = cmk(0.0, 0.0);
        d[rowmap ? rowmap[r] : r] = v;
    }
}

int jqr_extract(const PencilDev &P, double2 *dst, long ldd, const int *rowmap, hipStream_t s,
                int scatter) {
    int bx = (P.n + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_jqr_extract, dim3(bx, P.n), dim3(256), 0, s, P.n, P.Ft, P.ldft, P.perm,
                       P.rblk, P.pblk, rowmap, dst, ldd, scatter);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// ---------------------------------------------------------------------------
// Householder QR of G.
// ---------------------------------------------------------------------------
// One column step k, every trailing column in one launch: each workgroup
// forms the reflector H = I - v v^* / (||x|| (||x|| + |x_1|)) of column k
// (rows k..p-1; v = x + e^{i arg x_1} ||x|| e_1) from the column as stored,
// which no workgroup rewrites during the step, and applies it to its own
// column j > k; the workgroup of column k records R_kk = -e^{i arg x_1} ||x||.
template <int RC>
__device__ __forceinline__ void qr_col_step(const PencilDev &P, int k, int j, double *red);

// Column j of G's step k, workgroup bid of the window's column range.
template <int RC>
__device__ __forceinline__ void qr_step_body(const PencilDev *PD, const int *pre, int B, int k,
                                             int bid, int jw, double *red) {
    const int pk = find_pencil(pre, B, bid);
    const PencilDev P = PD[pk];
    if (!P.reduce || k >= P.n) return;
    const int j = pencil_local(pre, pk, bid) + jw;
    if (j < k) return;
    qr_col_step<RC>(P, k, j, red);
}

// Blocked form of G's QR (every pencil's p <= kQrRegRows): step k applies
// its reflector only to the columns of k's panel of kQrPanel columns,
// kQrPanel workgroups per pencil; k_qr_trail applies a finished panel's
// reflectors to the columns right of it.
template <int RC>
__device__ __forceinline__ void qr_panel_body(const PencilDev *PD, int B, int k, int bid,
                                              double *red) {
    const int pk = bid / kQrPanel;
    if (pk >= B) return;
    const PencilDev P = PD[pk];
    if (!P.reduce || k >= P.n) return;
    const int j = k - k % kQrPanel + bid % kQrPanel;
    if (j < k || j >= P.n) return;
    qr_col_step<RC>(P, k, j, red);
}

template <int RC>
__device__ __forceinline__ void qr_col_step(const PencilDev &P, int k, int j, double *red) {
    double2 *A = P.Gt;
    const long lda = P.ldgt;
    const int p = P.p;
    const double2 *x = A + (size_t)k * lda;
    double2 *y = A + (size_t)j * lda;
    if (p - k <= RC * kGridNT) {
        // both columns in registers, loaded together (rows k + tid + i *
        // kGridNT, the streaming loops' assignment)
        double2 xv[RC], yv[RC];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = k + (int)threadIdx.x + i * kGridNT;
            xv[i] = yv[i] = cmk(0.0, 0.0);
            if (r < p) {
                xv[i] = x[r];
                if (j != k) yv[i] = y[r];
            }
        }
        const double2 x1 = x[k];
        double s[1] = {0.0};
#pragma unroll
        for (int i = 0; i < RC; ++i)
            if (k + (int)threadIdx.x + i * kGridNT < p) s[0] += fnorm2(xv[i]);
        block_sum<1>(s, red);
        const double nrm = sqrt(s[0]);
        const double ax1 = sqrt(fnorm2(x1));
        const double2 ph = ax1 > 0.0 ? cmk(x1.x / ax1, x1.y / ax1) : cmk(1.0, 0.0);
        if (j == k) {
            if (threadIdx.x == 0) {
                P.qdiag[k] = nrm == 0.0 ? x1 : cscale(ph, -nrm);
                P.qnrm[k] = nrm;
            }
            return;
        }
        if (nrm == 0.0) return;
        const double cf = 1.0 / (nrm * (nrm + ax1));
        const double2 vk = cscale(ph, ax1 + nrm);
        double w[2] = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = k + (int)threadIdx.x + i * kGridNT;
            if (r < p) {
                const double2 a = r == k ? vk : xv[i], b = yv[i];
                w[0] += fdot_re(a, b);
                w[1] += fdot_im(a, b);
            }
        }
        block_sum<2>(w, red);
        const double2 tw = cmk(w[0] * cf, w[1] * cf);
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = k + (int)threadIdx.x + i * kGridNT;
            if (r < p) y[r] = csub(yv[i], fmul(r == k ? vk : xv[i], tw));
        }
        return;
    }
    double s[1] = {0.0};
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) s[0] += cnorm2(x[r]);
    block_sum<1>(s, red);
    const double nrm = sqrt(s[0]);
    const double2 x1 = x[k];
    const double ax1 = sqrt(cnorm2(x1));
    const double2 ph = ax1 > 0.0 ? cmk(x1.x / ax1, x1.y / ax1) : cmk(1.0, 0.0);
    if (j == k) {
        if (threadIdx.x == 0) {
            P.qdiag[k] = nrm == 0.0 ? x1 : cscale(ph, -nrm);
            P.qnrm[k] = nrm;
        }
        return;
    }
    if (nrm == 0.0) return;
    const double cf = 1.0 / (nrm * (nrm + ax1));  // 2 / (v^* v)
    const double2 vk = cscale(ph, ax1 + nrm);
    double w[2] = {0.0, 0.0};
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) {
        const double2 a = r == k ? vk : x[r], b = y[r];
        w[0] += a.x * b.x + a.y * b.y;
        w[1] += a.x * b.y - a.y * b.x;
    }
    block_sum<2>(w, red);
    const double2 tw = cmk(w[0] * cf, w[1] * cf);
    for (int r = k + threadIdx.x; r < p; r += blockDim.x) {
        const double2 a = r == k ? vk : x[r];
        y[r] = csub(y[r], cmul(a, tw));
    }
}

// A finished panel [ps, pe) of G's QR applied to the columns right of it:
// workgroup (g, pencil) holds columns pe + g kQrTrailCols .. + kQrTrailCols - 1,
// rows ps..p-1, in registers (row ps + tid + i kGridNT, p - ps <= kQrRegRows)
// and applies the panel's reflectors H_ps, ..., H_{pe-1} in order, each
// rebuilt from its stored column (rows > k), R's row k value x_1 and the
// recorded ||x||, as the step kernel builds it: w = v^* y, y <- y - v w / (||x||
// (||x|| + |x_1|)).  The columns are read and written once per panel instead
// of once per step.
__global__ __launch_bounds__(kGridNT) void k_qr_trail(const PencilDev *PD, int B, int ps, int pe) {
    constexpr int RC = kQrRegRows / kGridNT;
    constexpr int NC = kQrTrailCols;
    __shared__ double red[2 * NC * kGridNT / kWave];
    const int pk = blockIdx.y;
    if (pk >= B) return;
    const PencilDev P = PD[pk];
    if (!P.reduce || pe >= P.n) return;
    const int j0 = pe + (int)blockIdx.x * NC;
    if (j0 >= P.n) return;
    const int p = P.p;
    const long lda = P.ldgt;
    const GPtr<double2> A(P.Gt);
    const int tid = threadIdx.x;
    double2 y[NC][RC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = ps + tid + i * kGridNT;
            y[c][i] = (r < p && j0 + c < P.n) ? A.ld(r + (long)(j0 + c) * lda) : cmk(0.0, 0.0);
        }
    const int ke = pe < P.n ? pe : P.n;
    for (int k = ps; k < ke; ++k) {
        const double nrm = P.qnrm[k];
        if (nrm == 0.0) continue;
        const double2 x1 = A.ld(k + (long)k * lda);
        const double ax1 = sqrt(fnorm2(x1));
        const double2 ph = ax1 > 0.0 ? cmk(x1.x / ax1, x1.y / ax1) : cmk(1.0, 0.0);
        const double cf = 1.0 / (nrm * (nrm + ax1));
        const double2 vk = cscale(ph, ax1 + nrm);
        double2 v[RC];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = ps + tid + i * kGridNT;
            v[i] = r == k ? vk : ((r > k && r < p) ? A.ld(r + (long)k * lda) : cmk(0.0, 0.0));
        }
        double w[2 * NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            w[2 * c] = w[2 * c + 1] = 0.0;
#pragma unroll
            for (int i = 0; i < RC; ++i) {
                w[2 * c] += fdot_re(v[i], y[c][i]);
                w[2 * c + 1] += fdot_im(v[i], y[c][i]);
            }
        }
        block_sum<2 * NC>(w, red);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double2 tw = cmk(w[2 * c] * cf, w[2 * c + 1] * cf);
#pragma unroll
            for (int i = 0; i < RC; ++i) y[c][i] = csub(y[c][i], fmul(v[i], tw));
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < RC; ++i) {
            const int r = ps + tid + i * kGridNT;
            if (r < p && j0 + c < P.n) A.st(r + (long)(j0 + c) * lda, y[c][i]);
        }
}

// After the last step: R's diagonal in place and zeros below it.
__global__ void k_qr_settle(const PencilDev *PD) {
    const PencilDev P = PD[blockIdx.z];
    const int j = blockIdx.y;
    if (!P.reduce || j >= P.n) return;
    double2 *x = P.Gt + (size_t)j * P.ldgt;
    for (int r = j + blockIdx.x * blockDim.x + threadIdx.x; r < P.p; r += gridDim.x * blockDim.x)
        x[r] = r == j ? P.qdiag[j] : cmk(0.0, 0.0);
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

int jsplit_map(int rows, const int8_t *J, int *rowmap, int *nplus_dev, hipStream_t stream) {
    hipLaunchKernelGGL(k_jsplit_map, dim3(1), dim3(kOneNT), 0, stream, rows, J, rowmap, nplus_dev);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
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

// Input checks and ||G||_F^2.  Workgroup (x, j) writes its partial sum of
// column j to gnorm2[1 + 8 j + x]; k_check_sum adds the partials in one
// fixed order, so ||G||_F^2 does not depend on workgroup timing.
constexpr int kCheckSplit = 8;  // workgroups per column, at most

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
    if (threadIdx.x == 0) gnorm2[1 + (size_t)kCheckSplit * j + blockIdx.x] = g2[0];
}

// gnorm2[0] = the sum of the nx partials of each of the n columns: thread t
// adds columns t, t + 256, ... in order, then a fixed tree over the threads.
__global__ void k_check_sum(int n, int nx, double *gnorm2) {
    __shared__ double red[256 / kWave];
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        for (int x = 0; x < nx; ++x) v[0] += gnorm2[1 + (size_t)kCheckSplit * j + x];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) gnorm2[0] = v[0];
}

int check_inputs(int m, int n, int p, const double2 *F, long ldf, const int8_t *J,
                 const double2 *G, long ldg, int *flags, double *gnorm2, hipStream_t stream) {
    int rows = m > p ? m : p;
    int bx = (rows + 255) / 256;
    if (bx > kCheckSplit) bx = kCheckSplit;
    hipLaunchKernelGGL(k_check, dim3(bx, n), dim3(256), 0, stream, m, n, p, F, ldf, J, G, ldg,
                       flags, gnorm2);
    GHSVD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_check_sum, dim3(1), dim3(256), 0, stream, n, bx, gnorm2);
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
        const JqrState st = P.jst[0];
        out[2 * k] = st.status ? st.status : (st.k < P.n ? GHSVD_ERANK : 0);
        out[2 * k + 1] = st.n2x2;
    }
}

// After G's last column step: R's diagonal and the zeros below it.
static int qr_end(const BatchCtx &c, hipStream_t s) {
    int bx = (c.max_rows + 255) / 256;
    if (bx > 8) bx = 8;
    hipLaunchKernelGGL(k_qr_settle, dim3(bx, c.max_n, c.B), dim3(256), 0, s, c.dev);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// Section 5: the hyperbolic QR of F with its pivoting, and the QR of G.  The
// iteration sees G only through G^*G, so any square G_sq with G_sq^* G_sq =
// P2^T G^* G P2 serves: the triangular factor of G's unpivoted QR with its
// columns permuted by P2 afterwards (the caller gathers the columns of Gt by
// the permutation).  That QR needs no pivot decision; its column step it
// runs in the hyperbolic QR's step launch of iteration it.
int run_reduction(BatchCtx &c, std::vector<int> &status, std::vector<int> &n2x2,
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
        if ((rc = copy_cols(P.p, P.n, P.Gin, P.ldgin, P.Gt, P.ldgt, nullptr, s))) return rc;
        GHSVD_HIP(hipMemcpyAsync(P.Jw, P.Jin, (size_t)P.m, hipMemcpyDeviceToDevice, s));
    }
    // column windows: row w covers columns j >= w * step of each pencil; the
    // second table (from row kWinRows on) counts the step kernel's
    // workgroups, kStepCols columns each
    const int step = (c.max_n + kWinRows - 1) / kWinRows;
    const int rows = (c.max_n + step - 1) / step;
    const size_t pairs = (size_t)kWinRows * (B + 1);
    c.win.assign(2 * pairs, 0);
    for (int w = 0; w < rows; ++w)
        for (int k = 0; k < B; ++k) {
            const PencilDev &P = c.host[k];
            const int cols = P.reduce && P.n > w * step ? P.n - w * step : 0;
            const size_t e = (size_t)w * (B + 1) + k;
            c.win[e + 1] = c.win[e] + cols;
            c.win[pairs + e + 1] = c.win[pairs + e] + (cols + kStepCols - 1) / kStepCols;
        }
    GHSVD_HIP(hipMemcpyAsync(c.win_dev, c.win.data(), sizeof(int) * c.win.size(),
                             hipMemcpyHostToDevice, s));
    // rows per thread a window's step kernel keeps in registers: enough for
    // the longest trailing column of F (and, separately, of G) at the
    // window's first step
    std::vector<int> rows_f(rows, 0), rows_g(rows, 0);
    for (int w = 0; w < rows; ++w)
        for (const PencilDev &P : c.host) {
            if (!P.reduce || P.n <= w * step) continue;
            const int pf = (P.m - w * step + kGridNT - 1) / kGridNT;
            const int pg = (P.p - w * step + kGridNT - 1) / kGridNT;
            rows_f[w] = pf > rows_f[w] ? pf : rows_f[w];
            rows_g[w] = pg > rows_g[w] ? pg : rows_g[w];
        }
    int max_m = 0, max_p = 0;
    for (const PencilDev &P : c.host) {
        max_m = P.m > max_m ? P.m : max_m;
        if (P.reduce) max_p = P.p > max_p ? P.p : max_p;
    }
    // G's QR in panels when every column of G fits the trailing kernel's
    // registers (else one launch per column step over all trailing columns)
    const int qpanel = max_p <= kQrRegRows;
    const size_t jl_bytes = align_up((size_t)max_m, 16);
    hipLaunchKernelGGL(k_jqr_init, dim3(B), dim3(256), 0, s, c.dev);
    hipLaunchKernelGGL(k_jqr_colnorms, dim3(c.win[B]), dim3(kGridNT), 0, s, c.dev, c.win_dev, B, 0,
                       0);
    // At most max_n steps (fewer when 2x2 pivots occur; a pencil that has
    // finished has no workgroups left).  Three launches per step; the third
    // also carries G's column step it.
    for (int it = 0; it < c.max_n; ++it) {
        const int par = it & 1;
        const int w = it / step;
        const int *pw = c.win_dev + (size_t)w * (B + 1);
        const int tot = c.win[(size_t)w * (B + 1) + B];
        const int tot2 = c.win[pairs + (size_t)w * (B + 1) + B];
        const int jw = w * step;
        if (tot == 0) continue;
        // timed as one bracket: start of the first launch, end of the last
        hipEvent_t e0 = nullptr, e1 = nullptr;
        prof_take(kProfReduce, e0, e1);
        launch_ev(k_jqr_cross, dim3(tot), dim3(kGridNT), 0, s, e0, nullptr, c.dev, pw, B, par, jw);
        hipLaunchKernelGGL(k_jqr_cross2, dim3(tot), dim3(kGridNT), 0, s, c.dev, pw, B, par, jw);
        // 6 or 8 rows per thread only when every column fits: their register
        // counts lower the occupancy of the streaming paths.  Two F columns
        // per workgroup when F's columns fit 6 rows per thread (158 VGPRs,
        // three wavefronts per SIMD), else one (two columns at 8 rows would
        // leave two wavefronts per SIMD, and the streaming loops gain
        // nothing from sharing the pivot).
        const int rf = rows_f[w], rg = rows_g[w];
        const int cf = rf > 4 && rf <= 6 ? 1 : (rf > 6 && rf <= 8 ? 2 : (rf > 8 ? 3 : 0));
        const int cg = rg > 4 && rg <= 8 ? 1 : 0;
        decltype(&k_jqr_step<4, 4, 1>) const kinds[4][2] = {
            {k_jqr_step<4, 4, kStepCols>, k_jqr_step<4, 8, kStepCols>},
            {k_jqr_step<6, 4, kStepCols>, k_jqr_step<6, 8, kStepCols>},
            {k_jqr_step<8, 4, 1>, k_jqr_step<8, 8, 1>},
            {k_jqr_step<4, 4, 1>, k_jqr_step<4, 8, 1>}};
        auto step_k = kinds[cf][cg];
        const bool grouped = cf < 2;
        const int *pre_f = grouped ? pw + pairs : pw;
        const int tot_f = grouped ? tot2 : tot;
        const int gq = qpanel ? B * kQrPanel : tot;  // G's workgroups
        const bool trail = qpanel && (it % kQrPanel == kQrPanel - 1 || it == c.max_n - 1) &&
                           it - it % kQrPanel + kQrPanel < c.max_n;
        launch_ev(step_k, dim3(tot_f + gq), dim3(kGridNT), (uint32_t)jl_bytes, s, nullptr,
                  trail ? nullptr : e1, c.dev, pw, pre_f, B, par, tot_f, it, jw, qpanel);
        if (trail) {
            const int ps = it - it % kQrPanel, pe = ps + kQrPanel;
            launch_ev(k_qr_trail, dim3((c.max_n - pe + kQrTrailCols - 1) / kQrTrailCols, B),
                      dim3(kGridNT), 0, s, nullptr, e1, c.dev, B, ps, pe);
        }
        prof_done(kProfReduce, e0, e1);
    }
    hipLaunchKernelGGL(k_jqr_settle, dim3(B), dim3(256), 0, s, c.dev, c.max_n & 1);
    GHSVD_HIP(hipGetLastError());
    int rc = qr_end(c, s);
    if (rc) return rc;
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
