// phase4.hip -- the full GHSVD from a finished sweep stage (Phase 4,
// Section 7, with the outputs listed in Section 6.1).
//
// From the swept F' (rows 0..n_plus-1 carry J = +1, the rest -1), G' and the
// accumulated transformation Z':
//   Sigma_F' = diag(|f'_j^* J f'_j|^{1/2}), Sigma_G' = diag(||g'_j||),
//   Sigma_j = ((Sigma_F')_j^2 + (Sigma_G')_j^2)^{1/2},
//   U = F' Sigma_F'^{-1}, V = G' Sigma_G'^{-1},
//   Sigma_F = Sigma_F' Sigma^{-1}, Sigma_G = Sigma_G' Sigma^{-1},
//   Z = Z' Sigma^{-1}, X = Z^{-1},
// the inverse by LU with complete pivoting (P Z Q = L U, L unit lower
// triangular; among entries of equal modulus the pivot is the first in
// column-major order) and one pair of triangular solves per column of X,
// as the paper does with one solve per column in parallel.
//
// The factorization runs one column step per pair of launches: a single
// workgroup takes the pivot from the per-tile maxima, swaps the pivot row and
// column into place and scales the multipliers; then one workgroup per
// 64 x 64 tile of the trailing matrix applies the rank-one update and records
// the largest modulus of its updated tile for the next step.  The solves run
// one workgroup per column of X with the right-hand side in LDS.
#include "hz_common.hpp"

namespace ghsvd {

namespace {

constexpr int kP4Tile = 64;     // rows and columns of an update tile
constexpr int kP4Threads = 256;

struct TileMax {
    double v;   // largest |w|^2 of the tile (-1: empty)
    long idx;   // its column-major position col * n + row in the working matrix
};

// (v, idx) order: larger modulus first, then the earlier column-major position
__device__ __forceinline__ bool tm_better(double v, long i, double bv, long bi) {
    return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void block_tm(double &v, long &i, double *sv, long *si) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const long oi = __shfl_xor(i, off, kWave);
        if (tm_better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
    if (lane == 0) {
        sv[wid] = v;
        si[wid] = i;
    }
    __syncthreads();
    v = sv[0];
    i = si[0];
    for (int w = 1; w < nw; ++w)
        if (tm_better(sv[w], si[w], v, i)) {
            v = sv[w];
            i = si[w];
        }
    __syncthreads();
}

// Column statistics: s_f = |f'^* J f'|^{1/2}, s_g = ||g'||; flags bit 0 when
// either is zero, bit 1 when either is not finite.
__global__ __launch_bounds__(kP4Threads) void k_p4_stats(int m, int p, const double2 *F, long ldf,
                                                         int n_plus, const double2 *G, long ldg,
                                                         double *sf, double *sg, int *flags) {
    __shared__ double red[2 * kP4Threads / kWave];
    const int j = blockIdx.x;
    const double2 *f = F + (size_t)j * ldf;
    const double2 *g = G + (size_t)j * ldg;
    double v[2] = {0.0, 0.0};
    for (int r = threadIdx.x; r < m; r += blockDim.x) v[0] += (r < n_plus ? 1.0 : -1.0) * cnorm2(f[r]);
    for (int r = threadIdx.x; r < p; r += blockDim.x) v[1] += cnorm2(g[r]);
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        const double a = sqrt(fabs(v[0])), b = sqrt(v[1]);
        sf[j] = a;
        sg[j] = b;
        int bad = 0;
        if (!(a > 0.0) || !(b > 0.0)) bad |= 1;
        if (!isfinite(a) || !isfinite(b)) bad |= 2;
        if (bad) atomicOr(flags, bad);
    }
}

// U = F' / s_f, V = G' / s_g, W = Z' / Sigma (column j = blockIdx.y), and the
// normalized values sigma_f = s_f / Sigma, sigma_g = s_g / Sigma.
__global__ __launch_bounds__(kP4Threads) void k_p4_scale(int m, int p, int n, const double2 *F,
                                                         long ldf, const double2 *G, long ldg,
                                                         const double2 *Z, long ldz,
                                                         const double *sf, const double *sg,
                                                         double2 *U, long ldu, double2 *V, long ldv,
                                                         double2 *W, double *sigma_f,
                                                         double *sigma_g) {
    const int j = blockIdx.y;
    const double a = sf[j], b = sg[j];
    const double sig = sqrt(a * a + b * b);
    const int r0 = blockIdx.x * blockDim.x + threadIdx.x, rs = gridDim.x * blockDim.x;
    for (int r = r0; r < m; r += rs) {
        const double2 x = F[(size_t)j * ldf + r];
        U[(size_t)j * ldu + r] = cmk(x.x / a, x.y / a);
    }
    for (int r = r0; r < p; r += rs) {
        const double2 x = G[(size_t)j * ldg + r];
        V[(size_t)j * ldv + r] = cmk(x.x / b, x.y / b);
    }
    for (int r = r0; r < n; r += rs) {
        const double2 x = Z[(size_t)j * ldz + r];
        W[(size_t)j * n + r] = cmk(x.x / sig, x.y / sig);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sigma_f[j] = a / sig;
        sigma_g[j] = b / sig;
    }
}

// Tile maxima of |w|^2 over rows and columns k..n-1 of W (ld n), tiles of
// kP4Tile x kP4Tile; with upd, first the rank-one update of step k - 1
// (w_ij -= w_i,k-1 w_k-1,j for i, j >= k).
__global__ __launch_bounds__(kP4Threads) void k_p4_update(int n, int k, int upd, double2 *W,
                                                          TileMax *part) {
    __shared__ double sv[kP4Threads / kWave];
    __shared__ long si[kP4Threads / kWave];
    __shared__ double2 rowk[kP4Tile];
    const int nt = (n - k + kP4Tile - 1) / kP4Tile;
    const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;
    const int i0 = k + ti * kP4Tile, j0 = k + tj * kP4Tile;
    const int tid = threadIdx.x;
    const int kp = k - 1;
    if (upd && tid < kP4Tile) {
        const int j = j0 + tid;
        rowk[tid] = j < n ? W[(size_t)j * n + kp] : cmk(0.0, 0.0);
    }
    __syncthreads();
    double bv = -1.0;
    long bi = 0x7fffffffffffffffL;
    // thread t: row i0 + (t % 64), columns j0 + t / 64 + 4 c
    const int i = i0 + (tid % kP4Tile);
    const double2 lik = (upd && i < n) ? W[(size_t)kp * n + i] : cmk(0.0, 0.0);
    for (int c = tid / kP4Tile; c < kP4Tile; c += kP4Threads / kP4Tile) {
        const int j = j0 + c;
        if (i >= n || j >= n) continue;
        double2 *w = W + (size_t)j * n + i;
        double2 x = *w;
        if (upd) {
            const double2 u = rowk[c];
            x = csub(x, cmul(lik, u));
            *w = x;
        }
        const double v = cnorm2(x);
        const long idx = (long)j * n + i;
        if (tm_better(v, idx, bv, bi)) {
            bv = v;
            bi = idx;
        }
    }
    block_tm(bv, bi, sv, si);
    if (tid == 0) part[blockIdx.x] = TileMax{bv, bi};
}

// Pivot of step k from the tile maxima: swap row k with the pivot row and
// column k with the pivot column (whole rows and columns), record both, and
// divide the multipliers below the pivot by it.  flags bit 0 on a zero pivot.
__global__ __launch_bounds__(1024) void k_p4_pivot(int n, int k, double2 *W, const TileMax *part,
                                                   int *piv_r, int *piv_c, int *flags) {
    __shared__ double sv[1024 / kWave];
    __shared__ long si[1024 / kWave];
    const int nt = (n - k + kP4Tile - 1) / kP4Tile;
    double bv = -1.0;
    long bi = 0x7fffffffffffffffL;
    for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
        const TileMax m = part[t];
        if (tm_better(m.v, m.idx, bv, bi)) {
            bv = m.v;
            bi = m.idx;
        }
    }
    block_tm(bv, bi, sv, si);
    const int q = (int)(bi / n), pr = (int)(bi % n);
    if (!(bv > 0.0)) {
        if (threadIdx.x == 0) {
            atomicOr(flags, 1);
            piv_r[k] = k;
            piv_c[k] = k;
        }
        return;
    }
    // row swap k <-> pr over all columns, then column swap k <-> q over all rows
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double2 *a = W + (size_t)j * n;
        const double2 t = a[k];
        a[k] = a[pr];
        a[pr] = t;
    }
    __syncthreads();
    if (q != k) {
        double2 *a = W + (size_t)k * n, *b = W + (size_t)q * n;
        for (int r = threadIdx.x; r < n; r += blockDim.x) {
            const double2 t = a[r];
            a[r] = b[r];
            b[r] = t;
        }
    }
    __syncthreads();
    const double2 d = W[(size_t)k * n + k];
    const double dn = cnorm2(d);
    const double2 dinv = cmk(d.x / dn, -d.y / dn);  // 1 / d
    double2 *col = W + (size_t)k * n;
    for (int r = k + 1 + threadIdx.x; r < n; r += blockDim.x) col[r] = cmul(col[r], dinv);
    if (threadIdx.x == 0) {
        piv_r[k] = pr;
        piv_c[k] = q;
    }
}

// Column j of X = Q U^{-1} L^{-1} P e_j from P W Q = L U (W holds L below
// its diagonal and U on and above it): the row interchanges move e_j to
// e_r, then forward and back substitution in LDS, then the column
// interchanges place the entries.
__global__ __launch_bounds__(kP4Threads) void k_p4_solve(int n, const double2 *W, const int *piv_r,
                                                         const int *piv_c, double2 *X, long ldx) {
    extern __shared__ double2 y[];
    __shared__ int rsh;
    const int j = blockIdx.x;
    if (threadIdx.x == 0) {
        int r = j;
        for (int k = 0; k < n; ++k) {
            const int pk = piv_r[k];
            if (r == k) r = pk;
            else if (r == pk) r = k;
        }
        rsh = r;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = cmk(0.0, 0.0);
    __syncthreads();
    const int r = rsh;
    if (threadIdx.x == 0) y[r] = cmk(1.0, 0.0);
    __syncthreads();
    // L y = e_r (unit lower triangular): entries above r stay zero
    for (int t = r; t < n - 1; ++t) {
        const double2 yt = y[t];
        const double2 *l = W + (size_t)t * n;
        for (int i = t + 1 + threadIdx.x; i < n; i += blockDim.x) y[i] = csub(y[i], cmul(l[i], yt));
        __syncthreads();
    }
    // U w = y
    for (int t = n - 1; t >= 0; --t) {
        const double2 *u = W + (size_t)t * n;
        const double2 d = u[t];
        const double dn = cnorm2(d);
        const double2 wt = cmul(y[t], cmk(d.x / dn, -d.y / dn));
        __syncthreads();
        if (threadIdx.x == 0) y[t] = wt;
        for (int i = threadIdx.x; i < t; i += blockDim.x) y[i] = csub(y[i], cmul(u[i], wt));
        __syncthreads();
    }
    // X(:, j) = Q w: the column interchanges, applied in reverse order
    for (int k = n - 1; k >= 0; --k) {
        const int qk = piv_c[k];
        if (qk != k && threadIdx.x == 0) {
            const double2 t = y[k];
            y[k] = y[qk];
            y[qk] = t;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) X[(size_t)j * ldx + i] = y[i];
}

}  // namespace

}  // namespace ghsvd

using namespace ghsvd;

extern "C" int ghsvd_full(int m, int n, int p, const double *F, int ldf, int n_plus, const double *G,
                          int ldg, const double *Z, int ldz, double *U, int ldu, double *V, int ldv,
                          double *sigma_f, double *sigma_g, double *X, int ldx, void *stream) {
    if (n < 1 || m < n || p < n || n_plus < 0 || n_plus > m || ldf < m || ldg < p || ldz < n ||
        ldu < m || ldv < p || ldx < n || !F || !G || !Z || !U || !V || !sigma_f || !sigma_g || !X)
        return GHSVD_EINVAL;
    // the right-hand side of a solve lives in LDS
    if ((size_t)n * sizeof(double2) > 64 * 1024) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nt = (n + kP4Tile - 1) / kP4Tile;
    const size_t wbytes = align_up(sizeof(double2) * (size_t)n * n, 256);
    const size_t need = wbytes + align_up(sizeof(double) * 2 * (size_t)n, 256) +
                        align_up(sizeof(TileMax) * (size_t)nt * nt, 256) +
                        align_up(sizeof(int) * (2 * (size_t)n + 1), 256);
    char *buf = nullptr;
    if (hipMalloc(&buf, need) != hipSuccess) return GHSVD_EDEVICE;
    double2 *W = reinterpret_cast<double2 *>(buf);
    double *sf = reinterpret_cast<double *>(buf + wbytes);
    double *sg = sf + n;
    TileMax *part = reinterpret_cast<TileMax *>(buf + wbytes + align_up(sizeof(double) * 2 * (size_t)n, 256));
    int *piv_r = reinterpret_cast<int *>(reinterpret_cast<char *>(part) +
                                         align_up(sizeof(TileMax) * (size_t)nt * nt, 256));
    int *piv_c = piv_r + n;
    int *flags = piv_c + n;
    int rc = GHSVD_OK;
    int hflags = 0;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        return code;
    };
    if (hipMemsetAsync(flags, 0, sizeof(int), s) != hipSuccess) return fail(GHSVD_EDEVICE);
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    const double2 *G2 = reinterpret_cast<const double2 *>(G);
    const double2 *Z2 = reinterpret_cast<const double2 *>(Z);
    hipLaunchKernelGGL(k_p4_stats, dim3(n), dim3(kP4Threads), 0, s, m, p, F2, (long)ldf, n_plus, G2,
                       (long)ldg, sf, sg, flags);
    int bx = (m + kP4Threads - 1) / kP4Threads;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_p4_scale, dim3(bx, n), dim3(kP4Threads), 0, s, m, p, n, F2, (long)ldf, G2,
                       (long)ldg, Z2, (long)ldz, sf, sg, reinterpret_cast<double2 *>(U), (long)ldu,
                       reinterpret_cast<double2 *>(V), (long)ldv, W, sigma_f, sigma_g);
    if (hipGetLastError() != hipSuccess) return fail(GHSVD_EDEVICE);
    if (hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(GHSVD_EDEVICE);
    if (hflags & 2) return fail(GHSVD_ENONFINITE);
    if (hflags & 1) return fail(GHSVD_ERANK);
    // LU with complete pivoting: step k takes its pivot from the tile maxima
    // of rows and columns k..n-1, then updates them for step k + 1
    for (int k = 0; k < n; ++k) {
        const int t = (n - k + kP4Tile - 1) / kP4Tile;
        if (k == 0)
            hipLaunchKernelGGL(k_p4_update, dim3(t * t), dim3(kP4Threads), 0, s, n, 0, 0, W, part);
        hipLaunchKernelGGL(k_p4_pivot, dim3(1), dim3(1024), 0, s, n, k, W, part, piv_r, piv_c,
                           flags);
        if (k + 1 < n) {
            const int t1 = (n - k - 1 + kP4Tile - 1) / kP4Tile;
            hipLaunchKernelGGL(k_p4_update, dim3(t1 * t1), dim3(kP4Threads), 0, s, n, k + 1, 1, W,
                               part);
        }
    }
    hipLaunchKernelGGL(k_p4_solve, dim3(n), dim3(kP4Threads), sizeof(double2) * (size_t)n, s, n, W,
                       piv_r, piv_c, reinterpret_cast<double2 *>(X), (long)ldx);
    if (hipGetLastError() != hipSuccess) return fail(GHSVD_EDEVICE);
    if (hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(GHSVD_EDEVICE);
    rc = (hflags & 1) ? GHSVD_ERANK : GHSVD_OK;
    (void)hipFree(buf);
    return rc;
}
