// fast.hip -- the explicit-formation alternative of Section 4.5 for gfx950.
//
// The pencil is formed explicitly, H = F^* J F and S = G^* G (FP64 matrix
// cores, upper tiles computed and mirrored), and handed to a Cholesky-based
// generalized Hermitian eigensolver: S = R^* R (blocked, 64 x 64 tiles; the
// diagonal tile factored and inverted in LDS by one workgroup, the panel
// R_kj = R_kk^{-*} S_kj and the trailing update S_ij -= R_ki^* R_kj on MFMA),
// C = R^{-*} H R^{-1} by two blocked forward substitutions (the second reads
// its right-hand side W = R^{-*} H conjugate-transposed, since C = C^* =
// R^{-*} W^*), then C = V diag(lambda) V^* by blocked two-sided Jacobi
// (block columns of 16, the round-robin ordering over blocks; each block
// pair's 32 x 32 principal submatrix is diagonalized in LDS by one cyclic
// sweep of 2x2 rotations -- the full round-robin at the first block step of
// a sweep, only the pairs across the two blocks at the others -- and the
// accumulated rotations are applied two-sidedly to C, block by block on
// MFMA, and to the block columns of V), and X = R^{-1} V, eigenvalues
// ascending.
//
// A 2x2 rotation is applied when |c_pq| exceeds both eps sqrt(n)
// sqrt(|c_pp c_qq|) (the relative test of (6.12) with S = I) and eps sqrt(n)
// ||C||_F (C is stored explicitly, so its entries are only absolutely
// accurate and the relative test alone would chase rounding noise); the
// sweeps stop after one that applies no rotation.  The route squares the
// conditioning of G, so the caller's condition bound decides whether it is
// taken: when the Cholesky factor fails or (max r_ii / min r_ii)^2 exceeds
// the bound, the implicit HZ solve runs instead, with the caller's options.
#pragma clang fp contract(on)
#include "hz_common.hpp"

#include <cfloat>
#include <cmath>
#include <vector>

namespace ghsvd {
namespace {

constexpr int kFt = 64;    // tile of the formation, Cholesky and solves
constexpr int kJw = 16;    // Jacobi block width
constexpr int kJp = 32;    // Jacobi pivot order (two blocks)
typedef double fxv4d __attribute__((ext_vector_type(4)));

struct Acc {
    fxv4d re[2][2], im[2][2];
};

__device__ __forceinline__ void acc_zero(Acc &a) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            a.re[x][y] = fxv4d{0, 0, 0, 0};
            a.im[x][y] = fxv4d{0, 0, 0, 0};
        }
}

// acc += A B over k0 <= k < k0 + 4 for the 32 x 32 quarter (wi, wj) of a
// 64 x 64 complex tile; av, bv hold A[i][k] and B[k][j] of this lane (FP64
// MFMA 16x16x4: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k;
// result q of lane l at row l / 16 + 4 q, column l % 16 of its 16 x 16 tile).
__device__ __forceinline__ void mma4(const double2 (&av)[2], const double2 (&bv)[2], Acc &a) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            a.re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].x, bv[y].x, a.re[x][y], 0, 0, 0);
            a.re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[x].y, bv[y].y, a.re[x][y], 0, 0, 0);
            a.im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].x, bv[y].y, a.im[x][y], 0, 0, 0);
            a.im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].y, bv[y].x, a.im[x][y], 0, 0, 0);
        }
}

// acc += sum_{k < K} a(i, k) b(k, j) over the 64 x 64 tile, operands read
// straight from memory through the accessors (used where the inner
// dimension is one or a few tiles).
template <typename FA, typename FB>
__device__ __forceinline__ void tile_mma(FA a, FB b, int K, Acc &acc) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int wi = wv & 1, wj = wv >> 1, i16 = lane & 15, kq = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 4) {
        double2 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            av[t] = a(wi * 32 + t * 16 + i16, k0 + kq);
            bv[t] = b(k0 + kq, wj * 32 + t * 16 + i16);
        }
        mma4(av, bv, acc);
    }
}

// the accumulators into an LDS tile O[64][65]
__device__ __forceinline__ void acc_to_lds(const Acc &a, double2 (*O)[kFt + 1]) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int wi = wv & 1, wj = wv >> 1;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                O[wi * 32 + x * 16 + (lane >> 4) + 4 * q][wj * 32 + y * 16 + (lane & 15)] =
                    cmk(a.re[x][y][q], a.im[x][y][q]);
}

__device__ __forceinline__ void tri_decode(int e, int &i, int &j) {  // e -> i <= j
    int jj = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((jj + 1) * (jj + 2) / 2 <= e) ++jj;
    while (jj * (jj + 1) / 2 > e) --jj;
    j = jj;
    i = e - jj * (jj + 1) / 2;
}

// ---------------------------------------------------------------------------
// Formation: H = F^* J F (blockIdx.y = 0) and S = G^* G (blockIdx.y = 1), one
// upper tile (ti <= tj) per workgroup, rows staged through LDS 16 at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fx_form(int n, int m, int p, const double2 *F, int ldf,
                                                 const int8_t *J, const double2 *G, int ldg,
                                                 double2 *H, double2 *S) {
    __shared__ double2 lds[kFt * (kFt + 1)];
    double2(*As)[kFt + 1] = reinterpret_cast<double2(*)[kFt + 1]>(lds);            // [16][65]
    double2(*Bs)[kFt + 1] = reinterpret_cast<double2(*)[kFt + 1]>(lds + 16 * (kFt + 1));
    double2(*O)[kFt + 1] = reinterpret_cast<double2(*)[kFt + 1]>(lds);
    const bool isH = blockIdx.y == 0;
    const double2 *X = isH ? F : G;
    const int ld = isH ? ldf : ldg, rows = isH ? m : p;
    double2 *out = isH ? H : S;
    int ti, tj;
    tri_decode(blockIdx.x, ti, tj);
    const int ci = ti * kFt, cj = tj * kFt, tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid >> 6, wi = wv & 1, wj = wv >> 1;
    const int i16 = lane & 15, kq = lane >> 4;
    Acc acc;
    acc_zero(acc);
    for (int k0 = 0; k0 < rows; k0 += 16) {
        for (int e = tid; e < 16 * kFt; e += blockDim.x) {
            const int kk = e & 15, c = e >> 4, r = k0 + kk;
            const bool ok = r < rows;
            const double sg = (isH && ok) ? (J[r] > 0 ? 1.0 : -1.0) : 1.0;
            As[kk][c] = (ok && ci + c < n) ? X[(size_t)(ci + c) * ld + r] : cmk(0.0, 0.0);
            Bs[kk][c] = (ok && cj + c < n) ? cscale(X[(size_t)(cj + c) * ld + r], sg) : cmk(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            double2 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = cconj(As[ks + kq][wi * 32 + t * 16 + i16]);
                bv[t] = Bs[ks + kq][wj * 32 + t * 16 + i16];
            }
            mma4(av, bv, acc);
        }
        __syncthreads();
    }
    acc_to_lds(acc, O);
    __syncthreads();
    for (int e = tid; e < kFt * kFt; e += blockDim.x) {
        if (ti != tj) {
            const int i = e & 63, j = e >> 6;  // tile (ti, tj), column j
            if (ci + i < n && cj + j < n) out[(size_t)(cj + j) * n + ci + i] = O[i][j];
            const int jj = e & 63, ii = e >> 6;  // its mirror, column ci + ii
            if (ci + ii < n && cj + jj < n) out[(size_t)(ci + ii) * n + cj + jj] = cconj(O[ii][jj]);
        } else {
            const int i = e & 63, j = e >> 6;
            if (ci + i >= n || cj + j >= n) continue;
            double2 v = i <= j ? O[i][j] : cconj(O[j][i]);
            if (i == j) v.y = 0.0;
            out[(size_t)(cj + j) * n + ci + i] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Cholesky S = R^* R, R upper, in place in the upper tiles of S.
// ---------------------------------------------------------------------------

// Diagonal tile kt: factor in LDS, write R_kk (zero below its diagonal), its
// inverse Rinv[kt] (64 x 64 column-major, zero outside the valid block) and
// the diagonal entries.  flag[0] becomes 1 + the failing column on a pivot
// that is not positive and finite; later tiles then do nothing.
__global__ __launch_bounds__(256) void k_fx_chol_diag(int n, int kt, double2 *S, double2 *Rinv,
                                                      double *rdiag, int *flag) {
    __shared__ double2 A[kFt][kFt + 1];  // [row][col]
    __shared__ double2 Ri[kFt][kFt + 1];
    __shared__ double rinv;
    __shared__ int fail;
    if (*flag) return;
    const int tid = threadIdx.x, c0 = kt * kFt;
    const int nv = n - c0 < kFt ? n - c0 : kFt;
    for (int e = tid; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6;
        A[i][j] = (i < nv && j < nv && i <= j) ? S[(size_t)(c0 + j) * n + c0 + i] : cmk(0.0, 0.0);
        Ri[i][j] = cmk(0.0, 0.0);
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int c = 0; c < nv; ++c) {
        if (tid == 0) {
            const double d = A[c][c].x;
            if (!(d > 0.0) || !isfinite(d)) {
                fail = 1;
                *flag = 1 + c0 + c;
            } else {
                const double r = sqrt(d);
                A[c][c] = cmk(r, 0.0);
                rinv = 1.0 / r;
                rdiag[c0 + c] = r;
            }
        }
        __syncthreads();
        if (fail) return;
        for (int j = c + 1 + tid; j < nv; j += blockDim.x) A[c][j] = cscale(A[c][j], rinv);
        __syncthreads();
        const int rt = nv - c - 1, ntri = rt * (rt + 1) / 2;
        for (int e = tid; e < ntri; e += blockDim.x) {
            int ii, jj;
            tri_decode(e, ii, jj);
            const int i = c + 1 + ii, j = c + 1 + jj;
            A[i][j] = csub(A[i][j], cmulc(A[c][i], A[c][j]));
        }
        __syncthreads();
    }
    // inverse of the upper triangular R_kk, one column per thread: R x = e_j
    if (tid < nv) {
        const int j = tid;
        Ri[j][j] = cmk(1.0 / A[j][j].x, 0.0);
        for (int i = j - 1; i >= 0; --i) {
            double2 s = cmk(0.0, 0.0);
            for (int k = i + 1; k <= j; ++k) s = cadd(s, cmul(A[i][k], Ri[k][j]));
            Ri[i][j] = cscale(s, -1.0 / A[i][i].x);
        }
    }
    __syncthreads();
    for (int e = tid; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6;
        Rinv[(size_t)kt * kFt * kFt + e] = Ri[i][j];
        if (i < nv && j < nv) S[(size_t)(c0 + j) * n + c0 + i] = i <= j ? A[i][j] : cmk(0.0, 0.0);
    }
}

// Panel: R_{kt,tj} = R_kk^{-*} S_{kt,tj} for tj = kt + 1 + blockIdx.x.
__global__ __launch_bounds__(256) void k_fx_chol_panel(int n, int kt, double2 *S,
                                                       const double2 *Rinv, const int *flag) {
    __shared__ double2 O[kFt][kFt + 1];
    if (*flag) return;
    const int tj = kt + 1 + blockIdx.x, r0 = kt * kFt, c0 = tj * kFt;
    const double2 *Ri = Rinv + (size_t)kt * kFt * kFt;
    Acc acc;
    acc_zero(acc);
    tile_mma([&](int i, int k) { return cconj(Ri[(size_t)i * kFt + k]); },
             [&](int k, int j) {
                 return (r0 + k < n && c0 + j < n) ? S[(size_t)(c0 + j) * n + r0 + k] : cmk(0.0, 0.0);
             },
             kFt, acc);
    acc_to_lds(acc, O);
    __syncthreads();
    for (int e = threadIdx.x; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6;
        if (r0 + i < n && c0 + j < n) S[(size_t)(c0 + j) * n + r0 + i] = O[i][j];
    }
}

// Trailing update: S_{ti,tj} -= R_{kt,ti}^* R_{kt,tj}, kt < ti <= tj.
__global__ __launch_bounds__(256) void k_fx_chol_update(int n, int kt, double2 *S,
                                                        const int *flag) {
    __shared__ double2 O[kFt][kFt + 1];
    if (*flag) return;
    int a, b;
    tri_decode(blockIdx.x, a, b);
    const int ti = kt + 1 + a, tj = kt + 1 + b, r0 = kt * kFt, ci = ti * kFt, cj = tj * kFt;
    Acc acc;
    acc_zero(acc);
    tile_mma(
        [&](int i, int k) {
            return (r0 + k < n && ci + i < n) ? cconj(S[(size_t)(ci + i) * n + r0 + k]) : cmk(0.0, 0.0);
        },
        [&](int k, int j) {
            return (r0 + k < n && cj + j < n) ? S[(size_t)(cj + j) * n + r0 + k] : cmk(0.0, 0.0);
        },
        kFt, acc);
    acc_to_lds(acc, O);
    __syncthreads();
    for (int e = threadIdx.x; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6;
        if (ci + i < n && cj + j < n) {
            double2 &s = S[(size_t)(cj + j) * n + ci + i];
            s = csub(s, O[i][j]);
        }
    }
}

// ---------------------------------------------------------------------------
// Blocked triangular solves, one launch per block row `it`, one workgroup per
// tile column jt.  fwd = 1: R^* Y = B (block rows in increasing order),
// Y_it = R_it,it^{-*} (B_it - sum_{k < it} R_{k,it}^* Y_k); fwd = 0: R Y = B
// (decreasing order), Y_it = R_it,it^{-1} (B_it - sum_{k > it} R_{it,k} Y_k).
// B is read as is (Bt = 0) or conjugate-transposed (Bt = 1, B(i, j) =
// conj(Bsrc(j, i))).  Y may be Bsrc when Bt = 0 (in place).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fx_trsm(int n, int it, int fwd, int Bt, const double2 *R,
                                                 const double2 *Rinv, const double2 *Bsrc,
                                                 double2 *Y, const int *flag) {
    __shared__ double2 O[kFt][kFt + 1];
    if (*flag) return;
    const int nt = (n + kFt - 1) / kFt;
    const int jt = blockIdx.x, r0 = it * kFt, c0 = jt * kFt;
    Acc acc;
    acc_zero(acc);
    const int kb = fwd ? 0 : it + 1, ke = fwd ? it : nt;
    for (int kt = kb; kt < ke; ++kt) {
        const int k0 = kt * kFt;
        auto bY = [&](int k, int j) {
            return (k0 + k < n && c0 + j < n) ? Y[(size_t)(c0 + j) * n + k0 + k] : cmk(0.0, 0.0);
        };
        if (fwd)
            tile_mma([&](int i, int k) {
                         return (k0 + k < n && r0 + i < n) ? cconj(R[(size_t)(r0 + i) * n + k0 + k])
                                                           : cmk(0.0, 0.0);
                     },
                     bY, kFt, acc);
        else
            tile_mma([&](int i, int k) {
                         return (k0 + k < n && r0 + i < n) ? R[(size_t)(k0 + k) * n + r0 + i]
                                                           : cmk(0.0, 0.0);
                     },
                     bY, kFt, acc);
    }
    acc_to_lds(acc, O);
    __syncthreads();
    // O = B_it - O
    for (int e = threadIdx.x; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6, r = r0 + i, c = c0 + j;
        double2 b = cmk(0.0, 0.0);
        if (r < n && c < n) b = Bt ? cconj(Bsrc[(size_t)r * n + c]) : Bsrc[(size_t)c * n + r];
        O[i][j] = csub(b, O[i][j]);
    }
    __syncthreads();
    const double2 *Ri = Rinv + (size_t)it * kFt * kFt;
    acc_zero(acc);
    if (fwd)
        tile_mma([&](int i, int k) { return cconj(Ri[(size_t)i * kFt + k]); },
                 [&](int k, int j) { return O[k][j]; }, kFt, acc);
    else
        tile_mma([&](int i, int k) { return Ri[(size_t)k * kFt + i]; },
                 [&](int k, int j) { return O[k][j]; }, kFt, acc);
    __syncthreads();
    acc_to_lds(acc, O);
    __syncthreads();
    for (int e = threadIdx.x; e < kFt * kFt; e += blockDim.x) {
        const int i = e & 63, j = e >> 6;
        if (r0 + i < n && c0 + j < n) Y[(size_t)(c0 + j) * n + r0 + i] = O[i][j];
    }
}

// C <- (C + C^*) / 2 (diagonal real) and |c|^2 summed per column: workgroup
// j owns the entries (i, j) and (j, i), i <= j.
__global__ __launch_bounds__(256) void k_fx_sym(int n, double2 *C, double *part) {
    __shared__ double red[256 / kWave];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        double2 v;
        if (i == j) {
            v = cmk(C[(size_t)j * n + j].x, 0.0);
            C[(size_t)j * n + j] = v;
            s += v.x * v.x;
        } else {
            const double2 u = C[(size_t)j * n + i], l = C[(size_t)i * n + j];
            v = cscale(cadd(u, cconj(l)), 0.5);
            C[(size_t)j * n + i] = v;
            C[(size_t)i * n + j] = cconj(v);
            s += 2.0 * cnorm2(v);
        }
    }
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) t += red[w];
        part[j] = t;
    }
}

// ||C||_F from the column partials, in a fixed order; V = I.
__global__ __launch_bounds__(256) void k_fx_norm(int n, const double *part, double *nu) {
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) s += part[j];
    double v[1] = {s};
    __shared__ double lds[256 / kWave];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) *nu = sqrt(v[0]);
}

__global__ void k_fx_eye(int n, double2 *V) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (size_t)n * n) V[e] = cmk((e % n) == (e / n) ? 1.0 : 0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Blocked two-sided Jacobi on C.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int jcol(int n, int a, int b, int t) {  // pivot position -> column
    const int c = t < kJw ? a * kJw + t : b * kJw + t - kJw;
    return c < n ? c : -1;
}

// One workgroup per block pair of block step s: diagonalize the 32 x 32
// principal submatrix by one cyclic sweep, write the accumulated rotation
// Zh (32 x 32, column-major), the pair's flag (rotations applied) and add
// the count to *cnt.
__global__ __launch_bounds__(256) void k_fx_jinner(int n, int nb, int s, const double2 *C,
                                                   double2 *Zh, int *pflag, int *cnt,
                                                   const double *nu, const int *flag) {
    __shared__ double2 A[kJp][kJp + 1];
    __shared__ double2 Z[kJp][kJp + 1];
    __shared__ double rc[kJp / 2], rs[kJp / 2], l1[kJp / 2], l2[kJp / 2];
    __shared__ double2 re_[kJp / 2];
    __shared__ int rp[kJp / 2], rq[kJp / 2], ron[kJp / 2];
    __shared__ int col[kJp];
    if (*flag) return;
    const int k = blockIdx.x, tid = threadIdx.x;
    int a, b;
    rr_pair(nb, s, k, a, b);
    if (tid < kJp) col[tid] = jcol(n, a, b, tid);
    __syncthreads();
    for (int e = tid; e < kJp * kJp; e += blockDim.x) {
        const int i = e & 31, j = e >> 5;
        const int ci = col[i], cj = col[j];
        A[i][j] = (ci >= 0 && cj >= 0) ? C[(size_t)cj * n + ci] : cmk(0.0, 0.0);
        Z[i][j] = cmk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const double tol = DBL_EPSILON * sqrt((double)n);
    const double floor_ = tol * (*nu);
    const bool cross = s > 0;
    const int steps = cross ? kJw : kJp - 1;
    int count = 0;
    for (int st = 0; st < steps; ++st) {
        if (tid < kJp / 2) {
            int p, q;
            if (cross) {
                p = tid;
                q = kJw + (tid + st) % kJw;
            } else {
                rr_pair(kJp, st, tid, p, q);
            }
            int on = 0;
            if (col[p] >= 0 && col[q] >= 0) {
                const double x = A[p][p].x, y = A[q][q].x;
                const double2 c = A[p][q];
                const double ac = sqrt(cnorm2(c));
                if (ac > floor_ && ac > tol * sqrt(fabs(x * y))) {
                    const double tau = (y - x) / (2.0 * ac);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    const double cs = 1.0 / sqrt(1.0 + t * t);
                    rc[tid] = cs;
                    rs[tid] = t * cs;
                    re_[tid] = cscale(c, 1.0 / ac);
                    l1[tid] = x - t * ac;
                    l2[tid] = y + t * ac;
                    on = 1;
                    ++count;
                }
            }
            rp[tid] = p;
            rq[tid] = q;
            ron[tid] = on;
        }
        __syncthreads();
        // two-sided update of the 2x2 blocks (pair u rows, pair v columns),
        // one block per thread; the rotation R = [[cs, sn], [-sn conj(e), cs conj(e)]]
        {
            const int u = tid >> 4, v = tid & 15;
            const int p = rp[u], q = rq[u], pp = rp[v], qq = rq[v];
            const int onu = ron[u], onv = ron[v];
            if (onu || onv) {
                double2 b00 = A[p][pp], b01 = A[p][qq], b10 = A[q][pp], b11 = A[q][qq];
                if (onv) {  // columns: [x_p, x_q] R
                    const double cs = rc[v], sn = rs[v];
                    const double2 ec = cconj(re_[v]);
                    const double2 n00 = csub(cscale(b00, cs), cscale(cmul(b01, ec), sn));
                    const double2 n01 = cadd(cscale(b00, sn), cscale(cmul(b01, ec), cs));
                    const double2 n10 = csub(cscale(b10, cs), cscale(cmul(b11, ec), sn));
                    const double2 n11 = cadd(cscale(b10, sn), cscale(cmul(b11, ec), cs));
                    b00 = n00; b01 = n01; b10 = n10; b11 = n11;
                }
                if (onu) {  // rows: R^* [y_p; y_q]
                    const double cs = rc[u], sn = rs[u];
                    const double2 e = re_[u];
                    const double2 n00 = csub(cscale(b00, cs), cscale(cmul(e, b10), sn));
                    const double2 n01 = csub(cscale(b01, cs), cscale(cmul(e, b11), sn));
                    const double2 n10 = cadd(cscale(b00, sn), cscale(cmul(e, b10), cs));
                    const double2 n11 = cadd(cscale(b01, sn), cscale(cmul(e, b11), cs));
                    b00 = n00; b01 = n01; b10 = n10; b11 = n11;
                }
                if (u == v) {  // the pivot block becomes diag(l1, l2)
                    b00 = cmk(l1[u], 0.0);
                    b11 = cmk(l2[u], 0.0);
                    b01 = cmk(0.0, 0.0);
                    b10 = cmk(0.0, 0.0);
                }
                A[p][pp] = b00; A[p][qq] = b01; A[q][pp] = b10; A[q][qq] = b11;
            }
            // Z <- Z R for pair u, rows 2v and 2v + 1
            if (onu) {
                const double cs = rc[u], sn = rs[u];
                const double2 ec = cconj(re_[u]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = 2 * v + h;
                    const double2 zp = Z[i][p], zq = cmul(Z[i][q], ec);
                    Z[i][p] = csub(cscale(zp, cs), cscale(zq, sn));
                    Z[i][q] = cadd(cscale(zp, sn), cscale(zq, cs));
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < kJp * kJp; e += blockDim.x) Zh[(size_t)k * kJp * kJp + e] = Z[e & 31][e >> 5];
    // the count of the workgroup: one wavefront's lanes hold the pairs' counts
    __shared__ int total;
    if (tid == 0) total = 0;
    __syncthreads();
    if (tid < kJp / 2 && count) atomicAdd(&total, count);
    __syncthreads();
    if (tid == 0) {
        pflag[k] = total > 0;
        if (total) atomicAdd(cnt, total);
    }
}

// 32 x 32 complex product D = op(A) B on FP64 MFMA, operands and result in
// LDS: wavefront w forms the 16 x 16 tile (w & 1, w >> 1) of D; op(A) = A
// (conj_a = 0) or A^* (conj_a = 1).
__device__ __forceinline__ void mma32(const double2 (*A)[kJp + 1], const double2 (*Bm)[kJp + 1],
                                      double2 (*D)[kJp + 1], int conj_a) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int ti = wv & 1, tj = wv >> 1, i16 = lane & 15, kq = lane >> 4;
    fxv4d re = fxv4d{0, 0, 0, 0}, im = fxv4d{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < kJp; k0 += 4) {
        const double2 av = conj_a ? cconj(A[k0 + kq][ti * 16 + i16]) : A[ti * 16 + i16][k0 + kq];
        const double2 bv = Bm[k0 + kq][tj * 16 + i16];
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, im, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) D[ti * 16 + kq + 4 * q][tj * 16 + i16] = cmk(re[q], im[q]);
}

// The two-sided update of one block step in one pass: workgroups 0 ..
// npair^2 - 1 take the 32 x 32 block (pair u rows, pair v columns) of C to
// Zh_u^* C Zh_v (a side whose pair applied no rotation keeps the identity;
// a block neither side touches is skipped), so every entry of C is read and
// written once; the next npair * ceil(n / 32) workgroups take V's 32-row
// chunk r and pair v's columns to V Zh_v.  The pairs of a step are disjoint,
// so the blocks are independent.
__global__ __launch_bounds__(256) void k_fx_j2s(int n, int nb, int s, double2 *C, double2 *V,
                                                const double2 *Zh, const int *pflag,
                                                const int *flag) {
    __shared__ double2 X[kJp][kJp + 1];
    __shared__ double2 T[kJp][kJp + 1];
    __shared__ double2 Zu[kJp][kJp + 1];
    __shared__ double2 Zv[kJp][kJp + 1];
    __shared__ int colu[kJp], colv[kJp];
    if (*flag) return;
    const int npair = nb / 2, tid = threadIdx.x;
    const int nc = npair * npair;
    const bool isC = (int)blockIdx.x < nc;
    int u, v, r0 = 0;
    if (isC) {
        u = blockIdx.x % npair;
        v = blockIdx.x / npair;
    } else {
        const int e = blockIdx.x - nc;
        u = -1;
        v = e % npair;
        r0 = (e / npair) * kJp;
    }
    const int fu = u >= 0 ? pflag[u] : 0, fv = pflag[v];
    if (!fu && !fv) return;
    if (tid < kJp) {
        int a, b;
        rr_pair(nb, s, v, a, b);
        colv[tid] = jcol(n, a, b, tid);
        if (isC) {
            rr_pair(nb, s, u, a, b);
            colu[tid] = jcol(n, a, b, tid);
        } else {
            colu[tid] = r0 + tid < n ? r0 + tid : -1;  // plain rows of V
        }
    }
    __syncthreads();
    double2 *M = isC ? C : V;
    for (int e = tid; e < kJp * kJp; e += blockDim.x) {
        const int i = e & 31, j = e >> 5;
        const int ri = colu[i], cj = colv[j];
        X[i][j] = (ri >= 0 && cj >= 0) ? M[(size_t)cj * n + ri] : cmk(0.0, 0.0);
        if (fv) Zv[i][j] = Zh[(size_t)v * kJp * kJp + e];
        if (fu) Zu[i][j] = Zh[(size_t)u * kJp * kJp + e];
    }
    __syncthreads();
    double2(*R)[kJp + 1] = X;  // the current result
    if (fv) {
        mma32(X, Zv, T, 0);  // X Zh_v
        __syncthreads();
        R = T;
    }
    if (fu) {
        double2(*D)[kJp + 1] = R == X ? T : X;
        mma32(Zu, R, D, 1);  // Zh_u^* R
        __syncthreads();
        R = D;
    }
    for (int e = tid; e < kJp * kJp; e += blockDim.x) {
        const int i = e & 31, j = e >> 5;
        const int ri = colu[i], cj = colv[j];
        if (ri >= 0 && cj >= 0) M[(size_t)cj * n + ri] = R[i][j];
    }
}

// Eigenvalues ascending: rank of each diagonal entry (ties by index), then
// lambda and X's columns scattered to their ranks.
__global__ void k_fx_rank(int n, const double2 *C, int *rank, double *lam) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double v = C[(size_t)j * n + j].x;
    int r = 0;
    for (int i = 0; i < n; ++i) {
        const double u = C[(size_t)i * n + i].x;
        r += (u < v) || (u == v && i < j);
    }
    rank[j] = r;
    lam[r] = v;
}

__global__ void k_fx_scatter(int n, const double2 *Xv, const int *rank, double2 *X, int ldx) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int i = (int)(e % n), j = (int)(e / n);
    X[(size_t)rank[j] * ldx + i] = Xv[e];
}

struct FastWs {
    double2 *H, *S, *C, *V, *Rinv, *Zh;
    double *rdiag, *part, *nu, *lam;
    int *flag, *cnt, *pflag, *rank;
};

size_t fast_bytes(int n, FastWs *w, char *base) {
    const int nt = (n + kFt - 1) / kFt;
    int nb = (n + kJw - 1) / kJw;
    nb += nb & 1;
    Carver c{base, 0, ~size_t(0)};
    FastWs t;
    t.H = c.take<double2>((size_t)n * n);
    t.S = c.take<double2>((size_t)n * n);
    t.C = c.take<double2>((size_t)n * n);
    t.V = c.take<double2>((size_t)n * n);
    t.Rinv = c.take<double2>((size_t)nt * kFt * kFt);
    t.Zh = c.take<double2>((size_t)(nb / 2) * kJp * kJp);
    t.rdiag = c.take<double>(n);
    t.part = c.take<double>(n);
    t.nu = c.take<double>(1);
    t.lam = c.take<double>(n);
    t.flag = c.take<int>(4);
    t.cnt = t.flag + 1;
    t.pflag = c.take<int>(nb / 2);
    t.rank = c.take<int>(n);
    if (w) *w = t;
    return align_up(c.used, 256);
}

}  // namespace
}  // namespace ghsvd

using namespace ghsvd;

extern "C" size_t ghsvd_fast_workspace_size(int m, int n, int p, const ghsvd_options *fallback) {
    if (n < 1 || m < 1 || p < n) return 0;
    size_t need = fast_bytes(n, nullptr, nullptr);
    if (fallback) {
        const size_t hz = ghsvd_workspace_size(m, n, p, fallback);
        if (hz == 0) return 0;
        if (hz > need) need = hz;
    }
    return need;
}

extern "C" int ghsvd_solve_fast(int m, int n, int p, const double *F, int ldf,
                                const signed char *J, const double *G, int ldg, double *lambda,
                                double *X, int ldx, double cond_max, int max_sweeps, void *work,
                                size_t lwork, const ghsvd_options *fallback,
                                ghsvd_fast_info *info, void *stream) {
    ghsvd_fast_info loc{};
    ghsvd_fast_info *inf = info ? info : &loc;
    *inf = ghsvd_fast_info{};
    if (n < 1 || m < 1 || p < n || ldf < m || ldg < p || ldx < n) return inf->status = GHSVD_EINVAL;
    if (!F || !J || !G || !lambda || !X || !work) return inf->status = GHSVD_EINVAL;
    if (reinterpret_cast<uintptr_t>(work) & 255) return inf->status = GHSVD_EINVAL;
    if (lwork < ghsvd_fast_workspace_size(m, n, p, fallback)) return inf->status = GHSVD_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    FastWs w;
    fast_bytes(n, &w, static_cast<char *>(work));
    const int nt = (n + kFt - 1) / kFt;
    int nb = (n + kJw - 1) / kJw;
    nb += nb & 1;
    const int cap = max_sweeps > 0 ? max_sweeps : 60;
    const double2 *Fd = reinterpret_cast<const double2 *>(F);
    const double2 *Gd = reinterpret_cast<const double2 *>(G);
    GHSVD_HIP(hipMemsetAsync(w.flag, 0, 4 * sizeof(int), st));
    // H and S
    hipLaunchKernelGGL(k_fx_form, dim3(nt * (nt + 1) / 2, 2), dim3(256), 0, st, n, m, p, Fd, ldf,
                       reinterpret_cast<const int8_t *>(J), Gd, ldg, w.H, w.S);
    // S = R^* R
    for (int kt = 0; kt < nt; ++kt) {
        hipLaunchKernelGGL(k_fx_chol_diag, dim3(1), dim3(256), 0, st, n, kt, w.S, w.Rinv, w.rdiag,
                           w.flag);
        const int rest = nt - kt - 1;
        if (rest > 0) {
            hipLaunchKernelGGL(k_fx_chol_panel, dim3(rest), dim3(256), 0, st, n, kt, w.S, w.Rinv,
                               w.flag);
            hipLaunchKernelGGL(k_fx_chol_update, dim3(rest * (rest + 1) / 2), dim3(256), 0, st, n,
                               kt, w.S, w.flag);
        }
    }
    GHSVD_HIP(hipGetLastError());
    int hflag = 0;
    std::vector<double> rd(n);
    GHSVD_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    GHSVD_HIP(hipMemcpyAsync(rd.data(), w.rdiag, n * sizeof(double), hipMemcpyDeviceToHost, st));
    GHSVD_HIP(hipStreamSynchronize(st));
    double cond = 0.0;
    if (!hflag) {
        double lo = rd[0], hi = rd[0];
        for (int i = 1; i < n; ++i) {
            lo = rd[i] < lo ? rd[i] : lo;
            hi = rd[i] > hi ? rd[i] : hi;
        }
        cond = (hi / lo) * (hi / lo);
    }
    inf->cond_est = cond;
    if (hflag || !(cond <= cond_max)) {
        if (!fallback) return inf->status = GHSVD_ERANK;
        inf->path = GHSVD_PATH_HZ;
        const int rc = ghsvd_solve(m, n, p, F, ldf, J, G, ldg, lambda, X, ldx, work, lwork,
                                   fallback, &inf->hz, stream);
        inf->status = rc;
        return rc;
    }
    inf->path = GHSVD_PATH_FAST;
    // C = R^{-*} H R^{-1}: W = R^{-*} H in place of H, then C = R^{-*} W^*
    for (int it = 0; it < nt; ++it)
        hipLaunchKernelGGL(k_fx_trsm, dim3(nt), dim3(256), 0, st, n, it, 1, 0, w.S, w.Rinv, w.H,
                           w.H, w.flag);
    for (int it = 0; it < nt; ++it)
        hipLaunchKernelGGL(k_fx_trsm, dim3(nt), dim3(256), 0, st, n, it, 1, 1, w.S, w.Rinv, w.H,
                           w.C, w.flag);
    hipLaunchKernelGGL(k_fx_sym, dim3(n), dim3(256), 0, st, n, w.C, w.part);
    hipLaunchKernelGGL(k_fx_norm, dim3(1), dim3(256), 0, st, n, w.part, w.nu);
    hipLaunchKernelGGL(k_fx_eye, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256), 0, st,
                       n, w.V);
    GHSVD_HIP(hipGetLastError());
    // Jacobi sweeps
    const int npair = nb / 2, vch = (n + kJp - 1) / kJp;
    int sweeps = 0, converged = 0;
    long long rot = 0;
    while (sweeps < cap) {
        GHSVD_HIP(hipMemsetAsync(w.cnt, 0, sizeof(int), st));
        for (int s = 0; s < nb - 1; ++s) {
            hipLaunchKernelGGL(k_fx_jinner, dim3(npair), dim3(256), 0, st, n, nb, s, w.C, w.Zh,
                               w.pflag, w.cnt, w.nu, w.flag);
            hipLaunchKernelGGL(k_fx_j2s, dim3(npair * npair + npair * vch), dim3(256), 0, st, n,
                               nb, s, w.C, w.V, w.Zh, w.pflag, w.flag);
        }
        GHSVD_HIP(hipGetLastError());
        int hc = 0;
        GHSVD_HIP(hipMemcpyAsync(&hc, w.cnt, sizeof(int), hipMemcpyDeviceToHost, st));
        GHSVD_HIP(hipStreamSynchronize(st));
        ++sweeps;
        rot += hc;
        if (hc == 0) {
            converged = 1;
            break;
        }
    }
    inf->sweeps = sweeps;
    inf->rotations = rot;
    // X = R^{-1} V in place, then eigenvalues ascending
    for (int it = nt - 1; it >= 0; --it)
        hipLaunchKernelGGL(k_fx_trsm, dim3(nt), dim3(256), 0, st, n, it, 0, 0, w.S, w.Rinv, w.V,
                           w.V, w.flag);
    hipLaunchKernelGGL(k_fx_rank, dim3((n + 255) / 256), dim3(256), 0, st, n, w.C, w.rank, lambda);
    hipLaunchKernelGGL(k_fx_scatter, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256), 0,
                       st, n, w.V, w.rank, reinterpret_cast<double2 *>(X), ldx);
    GHSVD_HIP(hipGetLastError());
    return inf->status = converged ? GHSVD_OK : GHSVD_NOT_CONVERGED;
}
