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
// column-major order) and triangular solves with the identity as
// right-hand side (the paper solves the columns of X independently; here
// they are solved together, blocked).
//
// The factorization runs one launch per column step, with one workgroup per
// 64 x 64 tile of the trailing matrix.  Every workgroup takes the pivot from
// the tile maxima of the previous launch, reads its tile of the interchanged
// matrix through the two interchanges without moving any data, applies the
// rank-one update and writes the tile, with its largest modulus, to the other
// of two working matrices.  Rows and columns keep labels (their index in Z),
// so the multipliers and the pivot row of a step are stored at their labels
// and need no later interchanges; one gather puts L and U in the usual
// triangular layout.  The solves are blocked on 64 x 64 tiles (inverse
// diagonal blocks, then one launch per panel whose products run on the FP64
// MFMA) and store X through the row and column labels.
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

// Tile maxima of |w|^2 of the starting matrix W (ld n), tiles of
// kP4Tile x kP4Tile; workgroup 0 also gives every row and column its label
// (its index in W).
__global__ __launch_bounds__(kP4Threads) void k_p4_tilemax(int n, const double2 *W, TileMax *part,
                                                           int *rlab, int *clab) {
    __shared__ double sv[kP4Threads / kWave];
    __shared__ long si[kP4Threads / kWave];
    const int nt = (n + kP4Tile - 1) / kP4Tile;
    const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0)
        for (int r = tid; r < n; r += blockDim.x) {
            rlab[r] = r;
            clab[r] = r;
        }
    double bv = -1.0;
    long bi = 0x7fffffffffffffffL;
    // thread t: row ti * 64 + (t % 64), columns tj * 64 + t / 64 + 4 c
    const int i = ti * kP4Tile + (tid % kP4Tile);
    for (int c = tid / kP4Tile; c < kP4Tile; c += kP4Threads / kP4Tile) {
        const int j = tj * kP4Tile + c;
        if (i >= n || j >= n) continue;
        const double v = cnorm2(W[(size_t)j * n + i]);
        const long idx = (long)j * n + i;
        if (tm_better(v, idx, bv, bi)) {
            bv = v;
            bi = idx;
        }
    }
    block_tm(bv, bi, sv, si);
    if (tid == 0) part[blockIdx.x] = TileMax{bv, bi};
}

// Step k of the factorization, one launch.  Win holds rows and columns k..n-1
// of the working matrix after step k - 1 and pin their tile maxima (tiles
// anchored at k).  Every workgroup takes the pivot (pr, q) from pin itself.
// The interchanges of row k with row pr and of column k with column q are
// not made in memory: the interchanged matrix has at (i, j), i, j > k, the
// entry (rs(i), cs(j)) of Win, where rs swaps pr for k and cs swaps q for k.
// A workgroup updates one 64 x 64 tile of rows and columns k+1..n-1 of it by
// the rank-one term of step k and writes the tile, at the same positions, to
// Wout with its largest modulus for step k + 1.  Rows and columns carry
// labels (rl, cl; their index in the starting matrix), so the factors are
// stored by label: the multipliers of step k at Lt[label, k], the pivot row
// at Ut[k, label], the pivot at dg[k], the labels of the pivot's row and
// column at piv_r[k], piv_c[k].  flags bit 0 on a zero pivot; every step
// after it then finds a zero pivot too and writes nothing else.
constexpr int kP4Cols = kP4Tile * kWave / kP4Threads;  // tile columns per thread

// Tile `tile` of rows and columns k+1..n-1 (tiles of kP4Tile, column-major
// tile order): thread t holds row i0 + (t % 64), columns j0 + t / 64 + 4 c,
// read at the positions of the working matrix before the interchanges.
__device__ __forceinline__ void p4_load_tile(int n, int k, int tile, const double2 *Win,
                                             double2 (&x)[kP4Cols]) {
    const int nt1 = (n - k - 1 + kP4Tile - 1) / kP4Tile;
    const int ti = nt1 ? tile % nt1 : 0, tj = nt1 ? tile / nt1 : 0;
    const int i = k + 1 + ti * kP4Tile + ((int)threadIdx.x % kP4Tile);
    const int jt = k + 1 + tj * kP4Tile + (int)threadIdx.x / kP4Tile;
#pragma unroll
    for (int c = 0; c < kP4Cols; ++c) {
        const int j = jt + 4 * c;
        x[c] = (i < n && j < n) ? Win[(size_t)j * n + i] : cmk(0.0, 0.0);
    }
}

// The pivot of step k from the tile maxima pin (tiles anchored at k), the
// same in every workgroup: its modulus squared bv and position bi.
__device__ __forceinline__ void p4_find_pivot(int n, int k, const TileMax *pin, double *sv,
                                              long *si, double &bv, long &bi) {
    const int nt = (n - k + kP4Tile - 1) / kP4Tile;
    bv = -1.0;
    bi = 0x7fffffffffffffffL;
    for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
        const TileMax m = pin[t];
        if (tm_better(m.v, m.idx, bv, bi)) {
            bv = m.v;
            bi = m.idx;
        }
    }
    block_tm(bv, bi, sv, si);
}

// Step k on one tile, its entries x loaded by p4_load_tile and the pivot
// (bv, bi) known: the interchanged matrix has at (i, j), i, j > k, the entry
// (rs(i), cs(j)) of Win, rs swapping pr for k and cs swapping q for k, so
// only an entry in the pivot's row or column is read again.  Writes the
// updated tile to Wout and its largest modulus to *pout; the tiles of the
// first tile row and column also store the multipliers (Lt[label, k]) and
// the pivot row (Ut[k, label]) by label and the next labels, tile 0 the
// pivot (dg[k]) and its row and column labels.  A zero pivot sets flags
// bit 0 and leaves empty maxima, so that every later step finds one too.
__device__ __forceinline__ void p4_tile_update(
    int n, int k, int tile, double bv, long bi, double2 (&x)[kP4Cols], const double2 *Win,
    double2 *Wout, TileMax *pout, const int *rl_in, const int *cl_in, int *rl_out, int *cl_out,
    double2 *Lt, double2 *Ut, double2 *dg, int *piv_r, int *piv_c, int *flags, double *sv,
    long *si) {
    const int tid = threadIdx.x;
    if (!(bv > 0.0)) {
        if (tid == 0) {
            *pout = TileMax{-1.0, 0x7fffffffffffffffL};
            if (tile == 0) atomicOr(flags, 1);
        }
        return;
    }
    const int q = (int)(bi / n), pr = (int)(bi % n);
    const int nt1 = (n - k - 1 + kP4Tile - 1) / kP4Tile;
    const int ti = nt1 ? tile % nt1 : 0, tj = nt1 ? tile / nt1 : 0;
    const int i0 = k + 1 + ti * kP4Tile, j0 = k + 1 + tj * kP4Tile;
    const int i = i0 + (tid % kP4Tile);
    const int jt = j0 + tid / kP4Tile;
    const int rs = i == pr ? k : i;
    // the pivot, the multiplier of row i and the pivot row on this thread's
    // columns, all read at once
    const double2 d = Win[(size_t)q * n + pr];
    double2 l = i < n ? Win[(size_t)q * n + rs] : cmk(0.0, 0.0);
    double2 u[kP4Cols];
#pragma unroll
    for (int c = 0; c < kP4Cols; ++c) {
        const int j = jt + 4 * c;
        const int cs = j == q ? k : j;
        u[c] = j < n ? Win[(size_t)cs * n + pr] : cmk(0.0, 0.0);
        if (i < n && j < n && (i == pr || j == q)) x[c] = Win[(size_t)cs * n + rs];
    }
    const double dn = cnorm2(d);
    const double2 dinv = cmk(d.x / dn, -d.y / dn);  // 1 / d
    l = cmul(l, dinv);
    if (i < n && tj == 0 && tid < kP4Tile) {
        const int lab = rl_in[rs];
        Lt[(size_t)k * n + lab] = l;
        rl_out[i] = lab;
    }
    if (ti == 0 && tid < kP4Tile && j0 + tid < n) {
        const int j = j0 + tid;
        const int cs = j == q ? k : j;
        const int lab = cl_in[cs];
        Ut[(size_t)lab * n + k] = Win[(size_t)cs * n + pr];
        cl_out[j] = lab;
    }
    if (tile == 0 && tid == 0) {
        dg[k] = d;
        piv_r[k] = rl_in[pr];
        piv_c[k] = cl_in[q];
    }
    double tv = -1.0;
    long tix = 0x7fffffffffffffffL;
#pragma unroll
    for (int c = 0; c < kP4Cols; ++c) {
        const int j = jt + 4 * c;
        if (i >= n || j >= n) continue;
        const double2 y = csub(x[c], cmul(l, u[c]));
        Wout[(size_t)j * n + i] = y;
        const double v = cnorm2(y);
        const long idx = (long)j * n + i;
        if (tm_better(v, idx, tv, tix)) {
            tv = v;
            tix = idx;
        }
    }
    block_tm(tv, tix, sv, si);
    if (tid == 0) *pout = TileMax{tv, tix};
}

// Step k of the factorization, one launch with a workgroup per tile; the
// tile is read before the pivot is known.  (One cooperative launch for all
// steps, with a grid-wide barrier between them, took 2.5 times as long: the
// barrier across the chip costs more than the launch it saves.)
__global__ __launch_bounds__(kP4Threads) void k_p4_step(
    int n, int k, const double2 *Win, double2 *Wout, const TileMax *pin, TileMax *pout,
    const int *rl_in, const int *cl_in, int *rl_out, int *cl_out, double2 *Lt, double2 *Ut,
    double2 *dg, int *piv_r, int *piv_c, int *flags) {
    __shared__ double sv[kP4Threads / kWave];
    __shared__ long si[kP4Threads / kWave];
    double2 x[kP4Cols];
    p4_load_tile(n, k, blockIdx.x, Win, x);
    double bv;
    long bi;
    p4_find_pivot(n, k, pin, sv, si, bv, bi);
    p4_tile_update(n, k, blockIdx.x, bv, bi, x, Win, Wout, pout + blockIdx.x, rl_in, cl_in, rl_out,
                   cl_out, Lt, Ut, dg, piv_r, piv_c, flags, sv, si);
}

// P W Q = L U in the triangular layout (L below the diagonal, U on and
// above it, column c = blockIdx.x) from the factors stored by label:
// L(r, c) = Lt(piv_r[r], c) for r > c, U(r, c) = Ut(r, piv_c[c]) for r < c,
// U(c, c) = dg[c].
__global__ __launch_bounds__(kP4Threads) void k_p4_gather(int n, const double2 *Lt,
                                                          const double2 *Ut, const double2 *dg,
                                                          const int *piv_r, const int *piv_c,
                                                          double2 *LU, const int *flags) {
    if (*flags & 1) return;
    const int c = blockIdx.x;
    const double2 *lt = Lt + (size_t)c * n;
    const double2 *ut = Ut + (size_t)piv_c[c] * n;
    double2 *o = LU + (size_t)c * n;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        o[r] = r > c ? lt[piv_r[r]] : (r < c ? ut[r] : dg[c]);
}

// ---------------------------------------------------------------------------
// X = Q U^{-1} L^{-1} P by blocked triangular solves on 64 x 64 tiles.
// W1 = L^{-1} (lower triangular, the identity as right-hand side) and then
// W = U^{-1} W1; the interchanges only relabel: X[piv_c[c], piv_r[c']] =
// W[c, c'].  The diagonal blocks are inverted first (k_p4_dinv); panel k of
// either pass is one launch in which a workgroup multiplies its column tile
// of the panel's block row by the inverse diagonal block and, for a tile
// below (forward) or above (backward) the panel, subtracts the product with
// the panel's off-diagonal block of L or U.  The panel's block row is only
// read in the launch; the forward pass writes its finished block row to a
// second matrix, the backward pass straight into X.
// ---------------------------------------------------------------------------
constexpr int kTs = 64;  // tile order of the blocked solves

typedef double p4v4d __attribute__((ext_vector_type(4)));

// Inverse of diagonal block k of L (unit lower, blockIdx.y = 0) or of U
// (blockIdx.y = 1) of the triangular layout LU (ld n), 64 x 64, column-major,
// to D + (2 k + y) 64^2.  Past order n the block is the identity.  Thread t
// holds column t / 4 of the inverse, rows t % 4 + 4 r: the four threads of a
// column are adjacent lanes, so the substitution's pivot entry is a lane
// shuffle and no barrier is needed.
__global__ __launch_bounds__(256) void k_p4_dinv(int n, const double2 *LU, double2 *D) {
    __shared__ double2 Bk[kTs][kTs];  // the diagonal block, Bk[column][row]
    const int k = blockIdx.x, up = blockIdx.y;
    const int lane = threadIdx.x & (kWave - 1);
    const int j = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int b0 = k * kTs;
    const int nk = n - b0 < kTs ? n - b0 : kTs;
    for (int e = threadIdx.x; e < kTs * kTs; e += blockDim.x) {
        const int i = e % kTs, t = e / kTs;
        Bk[t][i] = (i < nk && t < nk) ? LU[(size_t)(b0 + t) * n + b0 + i] : cmk(0.0, 0.0);
    }
    __syncthreads();
    auto ent = [&](int i, int t) -> double2 { return Bk[t][i]; };
    double2 x[kTs / 4];
#pragma unroll
    for (int r = 0; r < kTs / 4; ++r) x[r] = cmk(q + 4 * r == j ? 1.0 : 0.0, 0.0);
    if (!up) {
        // L y = e_j: rows below t take the finished entry t
#pragma unroll 64
        for (int t = 0; t < kTs; ++t) {
            const double2 v = x[t >> 2];
            const double2 xt = cmk(__shfl(v.x, (lane & ~3) | (t & 3), kWave),
                                   __shfl(v.y, (lane & ~3) | (t & 3), kWave));
            if (t < nk) {
#pragma unroll
                for (int r = 0; r < kTs / 4; ++r) {
                    const int i = q + 4 * r;
                    if (i > t && i < nk) x[r] = csub(x[r], cmul(ent(i, t), xt));
                }
            }
        }
    } else {
        // U y = e_j: entry t is divided by u_tt, then rows above t take it
#pragma unroll 64
        for (int t = kTs - 1; t >= 0; --t) {
            const double2 v = x[t >> 2];
            double2 xt = cmk(__shfl(v.x, (lane & ~3) | (t & 3), kWave),
                             __shfl(v.y, (lane & ~3) | (t & 3), kWave));
            if (t < nk) {
                const double2 d = Bk[t][t];
                const double dn = cnorm2(d);
                xt = cmul(xt, cmk(d.x / dn, -d.y / dn));
                if (q == (t & 3)) x[t >> 2] = xt;
#pragma unroll
                for (int r = 0; r < kTs / 4; ++r) {
                    const int i = q + 4 * r;
                    if (i < t) x[r] = csub(x[r], cmul(ent(i, t), xt));
                }
            }
        }
    }
    double2 *o = D + (size_t)(2 * k + up) * kTs * kTs + (size_t)j * kTs;
#pragma unroll
    for (int r = 0; r < kTs / 4; ++r) o[q + 4 * r] = x[r];
}

// acc += A B for the 32 x 32 quarter (wi, wj) of a 64 x 64 complex product,
// a(i, k) and b(k, j) giving the operands (FP64 MFMA 16x16x4: A[i][k] from
// lane i + 16 k, B[k][j] from lane j + 16 k; result r of lane l at row
// l / 16 + 4 r, column l % 16 of its 16 x 16 tile).
template <typename FA, typename FB>
__device__ __forceinline__ void p4_mma64(FA a, FB b, int wi, int wj, int lane,
                                         p4v4d (&re)[2][2], p4v4d (&im)[2][2]) {
    const int i16 = lane & 15, kq = lane >> 4;
#pragma unroll 4
    for (int k0 = 0; k0 < kTs; k0 += 4) {
        double2 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            av[t] = a(wi * 32 + t * 16 + i16, k0 + kq);
            bv[t] = b(k0 + kq, wj * 32 + t * 16 + i16);
        }
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
            for (int tb = 0; tb < 2; ++tb) {
                re[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta].x, bv[tb].x, re[ta][tb], 0, 0, 0);
                re[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[ta].y, bv[tb].y, re[ta][tb], 0, 0, 0);
                im[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta].x, bv[tb].y, im[ta][tb], 0, 0, 0);
                im[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta].y, bv[tb].x, im[ta][tb], 0, 0, 0);
            }
    }
}

// One launch of panel k.  Forward (up = 0): workgroup (it, jt), it <
// nb - k, jt <= k (the tiles right of the diagonal stay zero), forms V =
// L_kk^{-1} Y(k, jt); it = 0 stores V as the finished Yf(k, jt), it > 0
// subtracts L(k + it, k) V from Y(k + it, jt).  Backward (up = 1):
// workgroup (it, jt), it <= k, forms V = U_kk^{-1} Yf(k, jt); it = 0 scatters
// V into X, it > 0 subtracts U(k - it, k) V from Yf(k - it, jt).  Entries
// past order n read as zero and are not written.
__global__ __launch_bounds__(256) void k_p4_panel(int n, int nb, int k, int up, const double2 *LU,
                                                  const double2 *D, double2 *Y, double2 *Yf,
                                                  const int *piv_r, const int *piv_c, double2 *X,
                                                  long ldx, const int *flags) {
    // one 64 x 64 tile in LDS: the right-hand side, then V, then the update
    __shared__ double2 Vs[kTs][kTs];  // [row][col]
    if (up && (*flags & 1)) return;  // the pivots are incomplete after a zero pivot
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
    const int wi = wv & 1, wj = wv >> 1;
    const int rows_it = up ? k + 1 : nb - k;
    const int it = blockIdx.x % rows_it, jt = blockIdx.x / rows_it;
    const int b0 = k * kTs, c0 = jt * kTs;
    const double2 *Dk = D + (size_t)(2 * k + up) * kTs * kTs;
    const double2 *src = up ? Yf : Y;  // the panel's block row
    // tile (row r0.., column c0..) of an n x n matrix to and from Vs, a column
    // of 64 rows per wavefront pass (coalesced)
    auto load_tile = [&](const double2 *M, int r0) {
        for (int e = tid; e < kTs * kTs; e += blockDim.x) {
            const int i = e % kTs, jj = e / kTs, r = r0 + i, c = c0 + jj;
            Vs[i][jj] = (r < n && c < n) ? M[(size_t)c * n + r] : cmk(0.0, 0.0);
        }
    };
    auto to_vs = [&](const p4v4d (&re)[2][2], const p4v4d (&im)[2][2]) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Vs[wi * 32 + a * 16 + (lane >> 4) + 4 * r][wj * 32 + b * 16 + (lane & 15)] =
                        cmk(re[a][b][r], im[a][b][r]);
    };
    auto dk = [&](int i, int kk) { return Dk[(size_t)kk * kTs + i]; };
    auto vs = [&](int kk, int jj) { return Vs[kk][jj]; };
    p4v4d re[2][2], im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            re[a][b] = p4v4d{0, 0, 0, 0};
            im[a][b] = p4v4d{0, 0, 0, 0};
        }
    load_tile(src, b0);
    __syncthreads();
    p4_mma64(dk, vs, wi, wj, lane, re, im);  // V = D_kk^{-1} (panel tile)
    __syncthreads();
    to_vs(re, im);
    __syncthreads();
    if (it == 0) {
        for (int e = tid; e < kTs * kTs; e += blockDim.x) {
            const int i = e % kTs, jj = e / kTs, row = b0 + i, col = c0 + jj;
            if (row >= n || col >= n) continue;
            if (!up) {
                Yf[(size_t)col * n + row] = Vs[i][jj];
            } else {
                const int xr = piv_c[row], xc = piv_r[col];
                if (xr >= 0 && xr < n && xc >= 0 && xc < n) X[(size_t)xc * ldx + xr] = Vs[i][jj];
            }
        }
        return;
    }
    const int t0 = up ? (k - it) * kTs : (k + it) * kTs;  // the block row updated
    auto off = [&](int i, int kk) {
        const int r = t0 + i, c = b0 + kk;
        return (r < n && c < n) ? LU[(size_t)c * n + r] : cmk(0.0, 0.0);
    };
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            re[a][b] = p4v4d{0, 0, 0, 0};
            im[a][b] = p4v4d{0, 0, 0, 0};
        }
    p4_mma64(off, vs, wi, wj, lane, re, im);  // (off-diagonal block) V
    __syncthreads();
    to_vs(re, im);
    __syncthreads();
    double2 *dst = up ? Yf : Y;
    for (int e = tid; e < kTs * kTs; e += blockDim.x) {
        const int i = e % kTs, jj = e / kTs, row = t0 + i, col = c0 + jj;
        if (row >= n || col >= n) continue;
        double2 *y = dst + (size_t)col * n + row;
        *y = csub(*y, Vs[i][jj]);
    }
}

// Y = I (ld n), Yf = 0
__global__ void k_p4_eye(int n, double2 *Y, double2 *Yf) {
    const int j = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        Y[(size_t)j * n + r] = cmk(r == j ? 1.0 : 0.0, 0.0);
        Yf[(size_t)j * n + r] = cmk(0.0, 0.0);
    }
}

}  // namespace

}  // namespace ghsvd

using namespace ghsvd;

namespace ghsvd {
namespace {

// Workspace of ghsvd_full: two working matrices (steps alternate between
// them), the factors by label, the column statistics, the pivots, two sets
// of tile maxima and of labels, the inverse diagonal blocks of the solves.
struct FullLayout {
    size_t wbytes, dbytes, gbytes, pbytes, ibytes, vbytes;
    size_t total() const { return 4 * wbytes + dbytes + gbytes + 2 * pbytes + ibytes + vbytes; }
};

FullLayout full_layout(int n) {
    const int nt = (n + kP4Tile - 1) / kP4Tile;
    const int nb = (n + kTs - 1) / kTs;  // tiles of the blocked solves
    FullLayout L;
    L.wbytes = align_up(sizeof(double2) * (size_t)n * n, 256);
    L.dbytes = align_up(sizeof(double) * 2 * (size_t)n, 256);
    L.gbytes = align_up(sizeof(double2) * (size_t)n, 256);
    L.pbytes = align_up(sizeof(TileMax) * (size_t)nt * nt, 256);
    L.ibytes = align_up(sizeof(int) * (6 * (size_t)n + 1), 256);
    L.vbytes = align_up(sizeof(double2) * 2 * (size_t)nb * kTs * kTs, 256);
    return L;
}

__global__ void k_p4_zero_flag(int *flags) {
    if (threadIdx.x == 0) flags[0] = 0;
}

}  // namespace
}  // namespace ghsvd

// the largest order ghsvd_full takes
static constexpr int kFullMaxN = 4096;

extern "C" size_t ghsvd_full_workspace_size(int n) {
    if (n < 1 || n > kFullMaxN) return 0;
    return full_layout(n).total();
}

extern "C" int ghsvd_full(int m, int n, int p, const double *F, int ldf, int n_plus, const double *G,
                          int ldg, const double *Z, int ldz, double *U, int ldu, double *V, int ldv,
                          double *sigma_f, double *sigma_g, double *X, int ldx, void *work,
                          size_t lwork, void *stream) {
    if (n < 1 || m < n || p < n || n_plus < 0 || n_plus > m || ldf < m || ldg < p || ldz < n ||
        ldu < m || ldv < p || ldx < n || !F || !G || !Z || !U || !V || !sigma_f || !sigma_g || !X)
        return GHSVD_EINVAL;
    if (n > kFullMaxN) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nt = (n + kP4Tile - 1) / kP4Tile;
    const int nb = (n + kTs - 1) / kTs;
    const FullLayout lay = full_layout(n);
    const size_t need = lay.total();
    char *buf = nullptr;
    bool owned = false;
    if (work) {
        if (lwork < need) return GHSVD_ENOMEM;
        if (reinterpret_cast<uintptr_t>(work) % 256) return GHSVD_EINVAL;
        buf = reinterpret_cast<char *>(work);
    } else {
        if (hipMalloc(&buf, need) != hipSuccess) return GHSVD_EDEVICE;
        owned = true;
    }
    char *at = buf;
    auto take = [&](size_t bytes) {
        char *r = at;
        at += bytes;
        return r;
    };
    const size_t wbytes = lay.wbytes, dbytes = lay.dbytes, gbytes = lay.gbytes;
    const size_t pbytes = lay.pbytes, ibytes = lay.ibytes, vbytes = lay.vbytes;
    double2 *Wb[2];
    Wb[0] = reinterpret_cast<double2 *>(take(wbytes));
    Wb[1] = reinterpret_cast<double2 *>(take(wbytes));
    double2 *Lt = reinterpret_cast<double2 *>(take(wbytes));
    double2 *Ut = reinterpret_cast<double2 *>(take(wbytes));
    double *sf = reinterpret_cast<double *>(take(dbytes));
    double *sg = sf + n;
    double2 *dg = reinterpret_cast<double2 *>(take(gbytes));
    TileMax *part[2];
    part[0] = reinterpret_cast<TileMax *>(take(pbytes));
    part[1] = reinterpret_cast<TileMax *>(take(pbytes));
    int *ib = reinterpret_cast<int *>(take(ibytes));
    int *piv_r = ib, *piv_c = ib + n;
    int *rl[2] = {ib + 2 * n, ib + 3 * n};
    int *cl[2] = {ib + 4 * n, ib + 5 * n};
    int *flags = ib + 6 * n;
    double2 *Dinv = reinterpret_cast<double2 *>(take(vbytes));  // inverse diagonal blocks
    double2 *W = Wb[0];
    int rc = GHSVD_OK;
    int hflags = 0;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        if (owned) (void)hipFree(buf);
        return code;
    };
    hipLaunchKernelGGL(k_p4_zero_flag, dim3(1), dim3(64), 0, s, flags);
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
    // LU with complete pivoting, one launch per step; step k reads the
    // working matrix, tile maxima and labels of parity k % 2 and writes
    // those of parity (k + 1) % 2
    hipLaunchKernelGGL(k_p4_tilemax, dim3(nt * nt), dim3(kP4Threads), 0, s, n, W, part[0], rl[0],
                       cl[0]);
    for (int k = 0; k < n; ++k) {
        const int t1 = (n - k - 1 + kP4Tile - 1) / kP4Tile;
        const int a = k & 1, b = a ^ 1;
        hipLaunchKernelGGL(k_p4_step, dim3(t1 > 0 ? t1 * t1 : 1), dim3(kP4Threads), 0, s, n, k,
                           Wb[a], Wb[b], part[a], part[b], rl[a], cl[a], rl[b], cl[b], Lt, Ut, dg,
                           piv_r, piv_c, flags);
    }
    hipLaunchKernelGGL(k_p4_gather, dim3(n), dim3(kP4Threads), 0, s, n, Lt, Ut, dg, piv_r, piv_c,
                       W, flags);
    // X = Q U^{-1} L^{-1} P: the diagonal blocks' inverses, then the panels of
    // the forward pass into Yf (Lt, free after the gather) with the working
    // right-hand side in the other working matrix, then the panels of the
    // backward pass into X
    double2 *Yw = Wb[1], *Yf = Lt;
    hipLaunchKernelGGL(k_p4_dinv, dim3(nb, 2), dim3(256), 0, s, n, W, Dinv);
    int ex = (n + 255) / 256;
    if (ex > 16) ex = 16;
    hipLaunchKernelGGL(k_p4_eye, dim3(ex, n), dim3(256), 0, s, n, Yw, Yf);
    double2 *X2 = reinterpret_cast<double2 *>(X);
    for (int k = 0; k < nb; ++k)
        hipLaunchKernelGGL(k_p4_panel, dim3((nb - k) * (k + 1)), dim3(256), 0, s, n, nb, k, 0, W,
                           Dinv, Yw, Yf, piv_r, piv_c, X2, (long)ldx, flags);
    for (int k = nb - 1; k >= 0; --k)
        hipLaunchKernelGGL(k_p4_panel, dim3((k + 1) * nb), dim3(256), 0, s, n, nb, k, 1, W, Dinv,
                           Yw, Yf, piv_r, piv_c, X2, (long)ldx, flags);
    if (hipGetLastError() != hipSuccess) return fail(GHSVD_EDEVICE);
    if (hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(GHSVD_EDEVICE);
    rc = (hflags & 1) ? GHSVD_ERANK : GHSVD_OK;
    if (owned) (void)hipFree(buf);
    return rc;
}
