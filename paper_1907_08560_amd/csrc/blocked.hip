// blocked.hip -- Level-2 blocked sweeps (Section 6.4, Block-Oriented inner
// level) with matrix-core (MFMA) Grams and block updates, and the complex
// FP32 warm-up stage with its FP64 hand-off.
//
// Block columns of width w (block b = columns [b w, min(b w + w, n)); nb =
// ceil(n / w) rounded up to even) are paired by the round-robin ordering; a
// block step handles nb / 2 disjoint block pairs at once in three kernels:
//   k_blk_gram   the block pivots H^ = F_C^* J F_C and S^ = G_C^* G_C
//                (order c <= 2w), as partial sums over 256-row chunks
//                (one workgroup per chunk; FP64 or FP32 MFMA 16x16x4);
//   k_blk_inner  one inner sweep (BO, Section 6.4.2) of the 2x2 step of
//                Section 6.1 over the c pivot columns in round-robin order,
//                applied two-sidedly to (H^, S^) held in LDS, accumulating
//                Z^ (c x c).  The 2x2 parameters are always FP64;
//   k_blk_update F_C <- F_C Z^, G_C <- G_C Z^, Z_C <- Z_C Z^ in place, per
//                64-row tile (MFMA), skipped when the inner sweep applied no
//                transformation (Section 6.4.3).
// The inner level works on the formed block pivots instead of factoring them
// into square J-factors first; the 2x2 step consumes only pivot entries, so
// the transformations are the same in exact arithmetic.  Convergence of the
// blocked stage: a block sweep whose inner sweeps applied no big
// transformation (Section 6.1.7).
#include <cmath>
#include <cstdlib>
#include <type_traits>

// Floating-point contraction is decided by the source expressions (a * b + c
// within one expression becomes one fused multiply-add), not by the code an
// expression is inlined into: the inner kernels and the look-ahead of their
// pivot wavefront evaluate the same expressions in different contexts and
// must round them the same way.
#pragma clang fp contract(on)

#include "hz_step.hpp"
#include "reduce.hpp"
#include "solver.hpp"

namespace ghsvd {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Both 16x16x4 forms take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  Result element r of lane l is D[row(l, r)][l % 16], with
// row = (l / 16) + 4 r for FP64 and 4 (l / 16) + r for FP32 (measured on
// gfx950 with an in-bounds probe).
template <>
struct Mfma<double> {
    using acc = v4d;
    using c2 = double2;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    using acc = v4f;
    using c2 = float2;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kGramChunk = 256;  // rows of one Gram partial

__device__ __forceinline__ int blk_width(int n, int w, int b) {
    const int c = n - b * w;
    return c < 0 ? 0 : (c > w ? w : c);
}

// Global column of pivot column cc (block a's columns, then block b's).
__device__ __forceinline__ int blk_col(int w, int a, int b, int ca, int cc) {
    return cc < ca ? a * w + cc : b * w + (cc - ca);
}

// Partial block-pivot Grams over one 256-row chunk of F (J-weighted) or G:
// P = X_C^* W X_C with X_C the c pivot columns.  Eight wavefronts each take
// 32 rows and read them straight into the operand layout of the 16x16x4
// MFMA (lane i + 16 k holds row k of pivot column i, for the column tiles
// 0..15 and 16..31): the same register is the A operand (conjugated,
// weighted) of one tile and the B operand of another.  Only the upper tiles
// of the Hermitian result are formed; the wavefronts' sums are added in LDS
// in a fixed order, and the lower tile is written as the conjugate
// transpose.  Padding columns (>= c) and rows past the end read as zero.
// The cross-wavefront sum runs in two halves (wavefronts 4-7 park their
// tiles, 0-3 add them to their own, then the four sums are added in order),
// so the LDS buffer holds four wavefronts' tiles and two workgroups share a
// CU.  In the FP32 warm-up the parked tiles and the first additions stay in
// FP32, the precision of the matrix-core sums themselves (24 KB instead of
// 48 KB of LDS, so two Gram workgroups fit beside an inner-sweep workgroup);
// the four half sums are added in FP64 as in the FP64 kernel.
constexpr int kGramWaves = 8;
constexpr int kGramHalf = kGramWaves / 2;

template <typename T, int PB>
__global__ __launch_bounds__(kWave * kGramWaves, 2) void k_blk_gram(const PencilDev *PD,
                                                                 const int *pre, const int *flag,
                                                                 int B, int step) {
    using C2 = typename Mfma<T>::c2;
    using ACC = typename Mfma<T>::acc;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NTD = PB / 16;              // column tiles
    constexpr int NT = NTD * (NTD + 1) / 2;   // upper output tiles
    constexpr int RW = kGramChunk / kGramWaves;  // rows per wavefront
    using RC2 = typename std::conditional<F32, float2, double2>::type;  // LDS partials
    __shared__ RC2 red[kGramHalf][NT][256];
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int local = pencil_local(pre, pk, blockIdx.x);
    const int KC = A.kf + A.kg;
    const int bpi = local / KC, kc = local % KC;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) return;
    const bool isF = kc < A.kf;
    const int r0 = (isF ? kc : kc - A.kf) * kGramChunk;
    const int rows = isF ? A.mr : A.pr;
    const long ld = isF ? A.ldf : A.ldg;
    const GPtr<C2> X(reinterpret_cast<const C2 *>(
        isF ? (F32 ? (const void *)A.F32 : (const void *)A.Fw)
            : (F32 ? (const void *)A.G32 : (const void *)A.Gw)));
    const int nplus = isF ? GPtr<int>(A.small).ld(1) : rows;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    GPtr<C2> col[NTD];
    bool okc[NTD];
#pragma unroll
    for (int t = 0; t < NTD; ++t) {
        const int cc = t * 16 + i16;
        okc[t] = cc < c;
        col[t] = X + (okc[t] ? (long)blk_col(A.w, a, b, ca, cc) * ld : 0L);
    }
    ACC acc_re[NT], acc_im[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        acc_re[q] = ACC{0, 0, 0, 0};
        acc_im[q] = ACC{0, 0, 0, 0};
    }
    const int rb = r0 + wv * RW + kq;
    C2 x[RW / 4][NTD];
#pragma unroll
    for (int ks = 0; ks < RW / 4; ++ks) {
        // every lane loads (a clamped, in-bounds address, so the value is
        // finite); padding is zeroed by a 0/1 factor where it is used
        const int r = rb + 4 * ks;
        const int rc = r < rows ? r : rows - 1;
#pragma unroll
        for (int t = 0; t < NTD; ++t) x[ks][t] = col[t].ld(rc);
    }
    // all loads are in flight before the first product: the products of
    // the first rows start as their loads complete, while the rest arrive
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < RW / 4; ++ks) {
        const int r = rb + 4 * ks;
        const bool okr = r < rows;
        const T wgt = (r >= nplus) ? T(-1) : T(1);
        T mb[NTD];
#pragma unroll
        for (int t = 0; t < NTD; ++t) mb[t] = (okc[t] && okr) ? T(1) : T(0);
        int q = 0;
#pragma unroll
        for (int ti = 0; ti < NTD; ++ti)
#pragma unroll
            for (int tj = ti; tj < NTD; ++tj, ++q) {
                const T fa = wgt * mb[ti];
                const T ar = fa * x[ks][ti].x, ai = fa * x[ks][ti].y;
                const T br = mb[tj] * x[ks][tj].x, bi = mb[tj] * x[ks][tj].y;
                // conj(a) b
                acc_re[q] = Mfma<T>::mma(ar, br, acc_re[q]);
                acc_re[q] = Mfma<T>::mma(ai, bi, acc_re[q]);
                acc_im[q] = Mfma<T>::mma(ar, bi, acc_im[q]);
                acc_im[q] = Mfma<T>::mma(-ai, br, acc_im[q]);
            }
    }
    if (wv >= kGramHalf) {
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                RC2 t;
                t.x = acc_re[q][r];
                t.y = acc_im[q][r];
                red[wv - kGramHalf][q][r * 64 + lane] = t;
            }
    }
    __syncthreads();
    if (wv < kGramHalf) {
#pragma unroll
        for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                RC2 &slot = red[wv][q][r * 64 + lane];
                slot.x = acc_re[q][r] + slot.x;
                slot.y = acc_im[q][r] + slot.y;
            }
    }
    __syncthreads();
    const GPtr<double2> P(A.part + ((size_t)bpi * KC + kc) * PB * PB);
    for (int e = tid; e < NT * 256; e += kWave * kGramWaves) {
        const int q = e / 256, rl = e % 256, r = rl / 64, ln = rl % 64;
        double2 sum = cmk((double)red[0][q][rl].x, (double)red[0][q][rl].y);
#pragma unroll
        for (int w2 = 1; w2 < kGramHalf; ++w2)
            sum = cadd(sum, cmk((double)red[w2][q][rl].x, (double)red[w2][q][rl].y));
        int ti = 0, tj = q;  // upper tile q -> (ti, tj)
        if (NTD == 2) {
            ti = q == 2 ? 1 : 0;
            tj = q == 0 ? 0 : 1;
        }
        const int i = ti * 16 + Mfma<T>::row(ln, r), j = tj * 16 + (ln & 15);
        P.st((long)j * PB + i, sum);
        if (ti != tj) P.st((long)i * PB + j, cconj(sum));
    }
}

// ---------------------------------------------------------------------------
// Block width 32: 64 pivot columns per block pair.
// ---------------------------------------------------------------------------
// Partial Grams over 128-row chunks.  The chunk is staged through LDS in two
// 64-row halves (the second half's loads are in flight while the first half
// is multiplied); wavefront t forms the upper 16x16 tile t of the 4x4 tile
// grid over all rows of the chunk, so no reduction across wavefronts is
// needed.  Tiles are written in the MFMA result layout; k_blk_gsum64 adds
// the chunks.  Padding columns (>= c) and rows past the end read as zero.
constexpr int kG64Chunk = 128;
constexpr int kG64Half = 64;
constexpr int kG64Tiles = 10;
constexpr int kG64Packed = 64 * 65 / 2;  // packed upper triangle of 64 x 64

// Upper tile t of the 4x4 grid: (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3)
// (2,2) (2,3) (3,3).
__device__ __forceinline__ void tile_of(int t, int &ti, int &tj) {
    ti = t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3));
    const int first = ti == 0 ? 0 : (ti == 1 ? 4 : (ti == 2 ? 7 : 9));
    tj = ti + (t - first);
}

// Packed upper triangle, column by column: entry (i, j), i <= j.
__device__ __forceinline__ int pk_idx(int i, int j) { return ((j * (j + 1)) >> 1) + i; }

template <typename T>
__global__ __launch_bounds__(kWave * kG64Tiles) void k_blk_gram64(const PencilDev *PD,
                                                                 const int *pre, const int *flag,
                                                                 int B, int step) {
    using C2 = typename Mfma<T>::c2;
    using ACC = typename Mfma<T>::acc;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int PB = 64;
    constexpr int NT = kWave * kG64Tiles;
    constexpr int PER = (kG64Half * PB + NT - 1) / NT;  // staged elements per thread
    __shared__ C2 Xs[2][kG64Half][PB + 1];
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int local = pencil_local(pre, pk, blockIdx.x);
    const int KC = A.kf + A.kg;
    const int bpi = local / KC, kc = local % KC;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) return;
    const bool isF = kc < A.kf;
    const int r0 = (isF ? kc : kc - A.kf) * kG64Chunk;
    const int rows = isF ? A.mr : A.pr;
    const long ld = isF ? A.ldf : A.ldg;
    const GPtr<C2> X(reinterpret_cast<const C2 *>(
        isF ? (F32 ? (const void *)A.F32 : (const void *)A.Fw)
            : (F32 ? (const void *)A.G32 : (const void *)A.Gw)));
    const int nplus = isF ? GPtr<int>(A.small).ld(1) : rows;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // element u of this thread in a half: column cc = e / 64, row e % 64
    C2 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = tid + u * NT, cc = e / kG64Half, r = r0 + e % kG64Half;
        const int rc = r < rows ? r : rows - 1;
        const long col = cc < c ? (long)blk_col(A.w, a, b, ca, cc) : 0L;
        v[u] = X.ld(col * ld + rc);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = tid + u * NT, cc = e / kG64Half, rl = e % kG64Half;
        if (e < kG64Half * PB) {
            const T m = (cc < c && r0 + rl < rows) ? T(1) : T(0);
            C2 x = v[u];
            x.x *= m;
            x.y *= m;
            Xs[0][rl][cc] = x;
        }
    }
    __syncthreads();
    // the second half's loads, in flight during the first half's products
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = tid + u * NT, cc = e / kG64Half, r = r0 + kG64Half + e % kG64Half;
        const int rc = r < rows ? r : rows - 1;
        const long col = cc < c ? (long)blk_col(A.w, a, b, ca, cc) : 0L;
        v[u] = X.ld(col * ld + rc);
    }
    int ti, tj;
    tile_of(wv, ti, tj);
    const int i16 = lane & 15, kq = lane >> 4;
    ACC acc_re = ACC{0, 0, 0, 0}, acc_im = ACC{0, 0, 0, 0};
#pragma unroll 4
    for (int ks = 0; ks < kG64Half / 4; ++ks) {
        const int rl = 4 * ks + kq;
        const T wgt = (r0 + rl >= nplus) ? T(-1) : T(1);
        const C2 xa = Xs[0][rl][ti * 16 + i16], xb = Xs[0][rl][tj * 16 + i16];
        const T ar = wgt * xa.x, ai = wgt * xa.y;
        // conj(a) b
        acc_re = Mfma<T>::mma(ar, xb.x, acc_re);
        acc_re = Mfma<T>::mma(ai, xb.y, acc_re);
        acc_im = Mfma<T>::mma(ar, xb.y, acc_im);
        acc_im = Mfma<T>::mma(-ai, xb.x, acc_im);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = tid + u * NT, cc = e / kG64Half, rl = e % kG64Half;
        if (e < kG64Half * PB) {
            const T m = (cc < c && r0 + kG64Half + rl < rows) ? T(1) : T(0);
            C2 x = v[u];
            x.x *= m;
            x.y *= m;
            Xs[1][rl][cc] = x;
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < kG64Half / 4; ++ks) {
        const int rl = 4 * ks + kq;
        const T wgt = (r0 + kG64Half + rl >= nplus) ? T(-1) : T(1);
        const C2 xa = Xs[1][rl][ti * 16 + i16], xb = Xs[1][rl][tj * 16 + i16];
        const T ar = wgt * xa.x, ai = wgt * xa.y;
        acc_re = Mfma<T>::mma(ar, xb.x, acc_re);
        acc_re = Mfma<T>::mma(ai, xb.y, acc_re);
        acc_im = Mfma<T>::mma(ar, xb.y, acc_im);
        acc_im = Mfma<T>::mma(-ai, xb.x, acc_im);
    }
    const GPtr<double2> P(A.part + (((size_t)bpi * KC + kc) * kG64Tiles + wv) * 256);
#pragma unroll
    for (int r = 0; r < 4; ++r) P.st(r * 64 + lane, cmk((double)acc_re[r], (double)acc_im[r]));
}

// Adds the chunk partials of upper tile t (blockIdx.y % 10) of H^ (chunks
// over F) or S^ (over G, blockIdx.y >= 10) of one block pair in chunk order,
// and writes the tile's entries on and above the diagonal, packed, for the
// inner sweep.
template <typename T>
__global__ __launch_bounds__(256) void k_blk_gsum64(const PencilDev *PD, const int *pre,
                                                    const int *flag, int B, int step) {
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int bpi = pencil_local(pre, pk, blockIdx.x);
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    if (blk_width(A.n, A.w, a) + blk_width(A.n, A.w, b) < 2) return;
    const int mat = blockIdx.y / kG64Tiles, t = blockIdx.y % kG64Tiles;
    const int KC = A.kf + A.kg;
    const int k0 = mat ? A.kf : 0, k1 = mat ? KC : A.kf;
    const int e = threadIdx.x, r = e / 64, ln = e % 64;
    const GPtr<double2> P(A.part);
    double2 sum = cmk(0.0, 0.0);
    for (int k = k0; k < k1; ++k) sum = cadd(sum, P.ld((((long)bpi * KC + k) * kG64Tiles + t) * 256 + e));
    int ti, tj;
    tile_of(t, ti, tj);
    const int i = ti * 16 + Mfma<T>::row(ln, r), j = tj * 16 + (ln & 15);
    if (i <= j) GPtr<double2>(A.gp).st(((long)bpi * 2 + mat) * kG64Packed + pk_idx(i, j), sum);
}

// r^* M c for one entry of a 2x2 block M = [[m00, m01], [m10, m11]]:
// x_a = m_a0 c0 + m_a1 c1, then conj(r0) x_0 + conj(r1) x_1.  The block
// update and the look-ahead of the pivot wavefront evaluate these same
// expressions, so the entries the look-ahead predicts equal the updated
// ones bit for bit.
__device__ __forceinline__ double2 mac2(double2 m0, double2 c0, double2 m1, double2 c1) {
    return cadd(cmul(m0, c0), cmul(m1, c1));
}
__device__ __forceinline__ double2 macc2(double2 r0, double2 x0, double2 r1, double2 x1) {
    return cadd(cmulc(r0, x0), cmulc(r1, x1));
}

// Threads of the inner kernel: one pivot wavefront, then one thread per 2x2
// block of (H^, S^) and one per 2x2 block of Z^.
template <int PB>
constexpr int inner_threads() {
    return kWave + PB * PB / 2;
}

// Pair ordering inside a block pivot of c columns (block a's columns first,
// then block b's).  Round-robin: the circle method of Section 6.3 over C = c
// rounded up to even, C - 1 steps of C / 2 slots, a pair meeting index c is
// a bye.  Cross (two full blocks of w columns): step s pairs column k of
// block a with column (k + s) mod w of block b, w steps of w slots.  Both
// directions are closed forms, so a slot's columns and a column's slot cost
// no memory access.
struct InnerOrder {
    int cross, C, w;
    __device__ int steps() const { return cross ? w : C - 1; }
    __device__ int slots() const { return cross ? w : C / 2; }
    __device__ void pair(int s, int k, int &p, int &q) const {
        if (cross) {
            int j = k + s;
            if (j >= w) j -= w;
            p = k;
            q = w + j;
        } else {
            rr_pair(C, s, k, p, q);
        }
    }
    // Slot of column x at step s, and its position in the pair (0: p, 1: q).
    // Every difference below lies in (-period, 2 period), so a conditional
    // add or subtract replaces the modulo.
    __device__ void where(int s, int x, int &slot, int &pos) const {
        if (cross) {
            int k = x - w - s;
            if (k < 0) k += w;
            slot = x < w ? x : k;
            pos = x < w ? 0 : 1;
            return;
        }
        const int M = C - 1;
        int partner;
        if (x == M) {
            slot = 0;
            partner = s;
        } else if (x == s) {
            slot = 0;
            partner = M;
        } else {
            int d = x - s;
            if (d < 0) d += M;
            if (d <= C / 2 - 1) {
                slot = d;
                partner = s - d;
                if (partner < 0) partner += M;
            } else {
                slot = M - d;
                partner = s + M - d;
                if (partner >= M) partner -= M;
            }
        }
        pos = x < partner ? 0 : 1;
    }
};

// Shared state of one inner step (double-buffered across steps).
template <int PB>
struct InnerStep {
    double2 z[PB / 2][4];  // Z' of each pair slot: z11, z21, z12, z22
    int act[PB / 2];       // 1: the slot applies its transformation
};

// The pivot wavefront's part of an inner step: the 2x2 steps of all pairs
// of inner step `is`.  (H, S) are the matrices before the update of step
// is - 1 (prev), which the other wavefronts are applying at the same time,
// and each pivot entry after that update is formed here from its 2x2 block
// and the two transformations that touch it.  Lane l forms entry kind
// e = l / 16 of pair k = l % 16 ((p, p), (q, q), (p, q)); lane k gathers its
// pair's six entries and runs the FP64 2x2 step.
// Look-ahead operands of lane l at inner step is (is >= 1), packed as bytes:
// x = rows r0, r1 and columns c0, c1 of the 2x2 block of step is - 1 that
// holds the lane's pivot entry; y = that block's row slot ki and position
// ii, column slot kj and position jj; y = kNoEntry when the lane forms no
// entry.  Filled once per launch from the closed-form ordering.
constexpr unsigned kNoEntry = 0xffffffffu;
// Lane of entry kind e of pair slot k in the pivot wavefront: k + 16 e, so
// that lane k reaches the other two kinds with the 16- and 32-lane swaps.
constexpr int kEntryStride = 16;
constexpr int kEntryLanes = 3 * kEntryStride;

// v from lane l + 16 (l < 16) and from lane l + 32 (l < 32).  Both sides of
// each swap are v, so the swap's second result is the shifted copy.
__device__ __forceinline__ double lane_plus16(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double lane_plus32(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)b[1], (int)a[1]);
}

// Step `is` follows step `prev` of the ordering: prev = is - 1 inside an
// inner sweep, prev = the last step when step 0 starts another inner sweep.
template <int PB>
__device__ __forceinline__ uint2 lookahead_entry(const InnerOrder &ord, int is, int prev, int l,
                                                 int c) {
    const int k = l % kEntryStride, e = l / kEntryStride;
    int pp = -1, qq = -1;
    if (k < ord.slots()) ord.pair(is, k, pp, qq);
    if (!(k < ord.slots() && qq < c && e < 3)) return make_uint2(0u, kNoEntry);
    const int i = (e == 1) ? qq : pp, j = (e == 0) ? pp : qq;
    int ki, ii, kj, jj, r0, r1, c0, c1;
    ord.where(prev, i, ki, ii);
    ord.where(prev, j, kj, jj);
    ord.pair(prev, ki, r0, r1);
    ord.pair(prev, kj, c0, c1);
    return make_uint2((unsigned)r0 | (unsigned)r1 << 8 | (unsigned)c0 << 16 | (unsigned)c1 << 24,
                      (unsigned)ki | (unsigned)ii << 8 | (unsigned)kj << 16 | (unsigned)jj << 24);
}

// Lane l of the pivot wavefront holds entry kind l / 16 of pair slot
// l % 16 (hv, sv); lane k < NP gathers its pair's (p,p), (q,q), (p,q) and
// runs the FP64 2x2 step (all lanes take part in the gather).
template <int PB, int F32>
__device__ __forceinline__ void pivot_finish(bool live, double2 hv, double2 sv, double tol, int crit,
                                             InnerStep<PB> &next, double &cv, double &ct,
                                             double &cbig, int *err) {
    constexpr int NP = PB / 2;
    const int l = threadIdx.x, k = l % kEntryStride;
    const double hpp = hv.x, hqq = lane_plus16(hv.x);
    const double hpq_r = lane_plus32(hv.x), hpq_i = lane_plus32(hv.y);
    const double spp = sv.x, sqq = lane_plus16(sv.x);
    const double spq_r = lane_plus32(sv.x), spq_i = lane_plus32(sv.y);
    if (l < NP) {
        int kind = kSkip;
        if (live) {
            Zp z;
            kind = hz_step_fast(hpp, hqq, cmk(hpq_r, hpq_i), spp, sqq, cmk(spq_r, spq_i), tol, crit,
                                z, F32);
            cv += 1.0;
            if (kind == GHSVD_ENONFINITE) atomicCAS(err, 0, GHSVD_ENONFINITE);
            if (kind < 0) kind = kSkip;  // dependent-looking pivot: left to the finish
            next.z[k][0] = z.z11;
            next.z[k][1] = z.z21;
            next.z[k][2] = z.z12;
            next.z[k][3] = z.z22;
            ct += kind > 0 ? 1.0 : 0.0;
            cbig += kind == kBig ? 1.0 : 0.0;
        }
        next.act[k] = kind > 0;
    }
}

// The pivot wavefront's part of inner step `is` >= 1: each lane forms its
// look-ahead entry (te: its operands, read from the table by the caller one
// step ahead) from the block entries before step is - 1 and that step's
// transformations, then the pairs' 2x2 steps run.
template <int PB, int F32>
__device__ __forceinline__ void inner_pivots(double tol, int crit, const double2 (*H)[PB + 1],
                                             const double2 (*S)[PB + 1],
                                             const InnerStep<PB> &prev, InnerStep<PB> &next,
                                             uint2 te, double &cv, double &ct, double &cbig,
                                             int *err) {
    constexpr int NP = PB / 2;
    static_assert(NP <= kEntryStride, "one lane per pair slot and entry kind");
    // this lane's entry; for lanes k < NP, whether pair k is live (its
    // (p,p) entry, formed by the lane itself, exists)
    const bool mine = te.y != kNoEntry, live = mine;
    double2 hv = cmk(0.0, 0.0), sv = cmk(0.0, 0.0);
    if (mine) {
        const double2 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0);
        const int r0 = te.x & 0xff, r1 = (te.x >> 8) & 0xff;
        const int c0 = (te.x >> 16) & 0xff, c1 = te.x >> 24;
        const int ki = te.y & 0xff, ii = (te.y >> 8) & 0xff;
        const int kj = (te.y >> 16) & 0xff, jj = te.y >> 24;
        // every operand is read at once (one LDS round trip); the
        // identity replaces an inactive slot's transformation by select
        const int ai = prev.act[ki], aj = prev.act[kj];
        const double2 za = prev.z[ki][2 * ii], zb = prev.z[ki][2 * ii + 1];
        const double2 zc = prev.z[kj][2 * jj], zd = prev.z[kj][2 * jj + 1];
        const double2 h00 = H[r0][c0], h01 = H[r0][c1], h10 = H[r1][c0], h11 = H[r1][c1];
        const double2 s00 = S[r0][c0], s01 = S[r0][c1], s10 = S[r1][c0], s11 = S[r1][c1];
        // column ii of Z'_ki, column jj of Z'_kj
        const double2 ra = ai ? za : (ii ? zero : one), rb = ai ? zb : (ii ? one : zero);
        const double2 ca = aj ? zc : (jj ? zero : one), cb = aj ? zd : (jj ? one : zero);
        hv = macc2(ra, mac2(h00, ca, h01, cb), rb, mac2(h10, ca, h11, cb));
        sv = macc2(ra, mac2(s00, ca, s01, cb), rb, mac2(s10, ca, s11, cb));
    }
    pivot_finish<PB, F32>(live, hv, sv, tol, crit, next, cv, ct, cbig, err);
}

// One inner sweep over the block pivot (H^, S^) in LDS, software-pipelined.
// While wavefront 0 computes the 2x2 steps of inner step s + 1 (with the
// pivot entries predicted from the block entries before step s and step s's
// transformations), the other threads apply step s: one thread per 2x2
// block (rows of pair k, columns of pair k') does H <- Z_k^* H Z_k' and
// S <- Z_k^* S Z_k' from one buffer into the other, and one thread per 2x2
// block does Zs <- Zs Z_k' in place.  The pairs of a step are disjoint, so
// the blocks are independent.  Pair slots whose second column is a bye or
// padding (>= c) carry the identity; padding entries are zero and stay so.
// mode GHSVD_INNER_CROSS: block steps after the first of a sweep visit only
// the w^2 pairs across the two blocks (InnerOrder cross); the first block
// step of a sweep, where every block appears once, visits all pairs, so that
// each pair of columns is visited once per sweep.  mode GHSVD_INNER_FB (the
// Full Block variant of Section 6.4.2): round-robin inner sweeps follow one
// another, the step after the last of a sweep being step 0 of the next, until
// an inner sweep applies no transformation at all (big or small: Section
// 6.1.7 has inner levels count every transformation for stopping) or
// kFbSweeps have run.  The pivot wavefront, which forms the pivots of the
// next step while the last step of a sweep is applied, decides from the
// sweep's transformation count whether there is a next sweep and posts the
// decision for the whole workgroup.
constexpr int kFbSweeps = 30;  // C_max of the FB inner level

template <int PB, int F32, int FB>
__global__ __launch_bounds__(inner_threads<PB>()) void k_blk_inner(const PencilDev *PD,
                                                                   const int *pre, const int *flag,
                                                                   int B, int crit, int step,
                                                                   int mode) {
    constexpr int NP = PB / 2;   // pivot pair slots per inner step
    constexpr int NB = NP * NP;  // 2x2 blocks
    __shared__ double2 H[2][PB][PB + 1];
    __shared__ double2 S[2][PB][PB + 1];
    __shared__ double2 Zs[PB][PB + 1];
    __shared__ InnerStep<PB> st[2];
    __shared__ uint2 tab[PB][kEntryLanes];  // look-ahead operands per inner step and lane
    __shared__ int more[2];                 // FB: another inner sweep follows (by parity)
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int bpi = pencil_local(pre, pk, blockIdx.x);
    const int tid = threadIdx.x;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) {
        if (tid == 0) GPtr<int>(A.ntr).st(bpi, 0);
        return;
    }
    // the latency-critical pivot wavefront issues first
    if (tid < kWave) __builtin_amdgcn_s_setprio(3);
    InnerOrder ord;
    ord.cross = !FB && mode == GHSVD_INNER_CROSS && step > 0 && ca == NP && cb == NP;
    ord.C = c + (c & 1);
    ord.w = NP;
    const int nsteps = ord.steps(), nsl = ord.slots();
    constexpr int max_isw = FB ? kFbSweeps : 1;  // FB: mode is GHSVD_INNER_FB
    const int KC = A.kf + A.kg;
    const GPtr<double2> P(A.part + (size_t)bpi * KC * PB * PB);
    const double tol = (F32 ? 0x1p-23 : 0x1p-52) * sqrt((double)c);
    double cv = 0.0, ct = 0.0, cbig = 0.0;
    if (tid < kWave) {
        // inner step 0 straight from the partial Grams, summed in the chunk
        // order of the LDS fill below (so the entries are the same bits),
        // while the other wavefronts fill LDS
        const int k = tid % kEntryStride, e = tid / kEntryStride;
        int pp = -1, qq = -1;
        if (k < nsl) ord.pair(0, k, pp, qq);
        const bool live = k < nsl && qq < c;
        double2 hv = cmk(0.0, 0.0), sv = cmk(0.0, 0.0);
        if (live && e < 3) {
            const int i = (e == 1) ? qq : pp, j = (e == 0) ? pp : qq;
            const long off = i + (long)PB * j;
#pragma unroll 4
            for (int kk = 0; kk < A.kf; ++kk) hv = cadd(hv, P.ld((long)kk * PB * PB + off));
#pragma unroll 4
            for (int kk = A.kf; kk < KC; ++kk) sv = cadd(sv, P.ld((long)kk * PB * PB + off));
        }
        pivot_finish<PB, F32>(live, hv, sv, tol, crit, st[0], cv, ct, cbig, &A.st->err);
    } else {
        const int t0 = tid - kWave, nt = inner_threads<PB>() - kWave;
        for (int idx = t0; idx < PB * PB; idx += nt) {
            const int i = idx % PB, j = idx / PB;
            double2 h = cmk(0.0, 0.0), s = cmk(0.0, 0.0);
            // partials summed in chunk order; unrolled so the loads issue together
#pragma unroll 4
            for (int k = 0; k < A.kf; ++k) h = cadd(h, P.ld((long)k * PB * PB + idx));
#pragma unroll 4
            for (int k = A.kf; k < KC; ++k) s = cadd(s, P.ld((long)k * PB * PB + idx));
            H[0][i][j] = h;
            S[0][i][j] = s;
            Zs[i][j] = cmk(i == j ? 1.0 : 0.0, 0.0);
        }
        for (int idx = t0; idx < (nsteps - 1) * kEntryLanes; idx += nt) {
            const int is = 1 + idx / kEntryLanes, l = idx % kEntryLanes;
            tab[is][l] = lookahead_entry<PB>(ord, is, is - 1, l, c);
        }
        // FB: row 0 holds step 0 of a following inner sweep
        if (max_isw > 1)
            for (int l = t0; l < kEntryLanes; l += nt)
                tab[0][l] = lookahead_entry<PB>(ord, 0, nsteps - 1, l, c);
    }
    __syncthreads();
    // look-ahead operands of the next inner step, read one step ahead
    uint2 te = make_uint2(0u, kNoEntry);
    if (tid < kWave && tid < kEntryLanes) {
        if (nsteps > 1) te = tab[1][tid];
        else if (max_isw > 1) te = tab[0][tid];
    }
    double cmark = 0.0;  // ct at the end of the previous inner sweep
    int g = 0;           // inner steps so far (parity of the H, S and step buffers)
    for (int isw = 0;; ++isw) {
    for (int s = 0; s < nsteps; ++s, ++g) {
        const int cur = g & 1, nxt = cur ^ 1;
        const InnerStep<PB> &now = st[cur];
        if (tid < kWave) {
            bool go = s + 1 < nsteps;
            if (!go && isw + 1 < max_isw) {
                // the pivots of this sweep's last step are in ct: another
                // sweep follows when the sweep applied any transformation,
                // big or small (inner levels count them all for stopping)
                const double sa = wave_sum(ct - cmark);
                cmark = ct;
                go = sa > 0.0;
                if (tid == 0) more[isw & 1] = go;
            }
            if (go) {
                inner_pivots<PB, F32>(tol, crit, H[cur], S[cur], now, st[nxt], te, cv, ct, cbig,
                                      &A.st->err);
                const int s2 = (s + 2) % nsteps;
                te = ((s + 2 < nsteps || max_isw > 1) && tid < kEntryLanes)
                         ? tab[s2][tid]
                         : make_uint2(0u, kNoEntry);
            }
        } else {
            const double2 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0);
            const int t = tid - kWave;
            const int blk = t < NB ? t : t - NB;
            const int kr = blk % NP, kc = blk / NP;  // row pair, column pair
            if (kr < nsl && kc < nsl) {
                int p1, q1, p2, q2;
                ord.pair(s, kr, p1, q1);
                ord.pair(s, kc, p2, q2);
                const bool ar = now.act[kr], ac = now.act[kc];
                double2 c11 = one, c21 = zero, c12 = zero, c22 = one;
                if (ac) {
                    c11 = now.z[kc][0];
                    c21 = now.z[kc][1];
                    c12 = now.z[kc][2];
                    c22 = now.z[kc][3];
                }
                if (t < NB) {
                    const double2 h11 = H[cur][p1][p2], h12 = H[cur][p1][q2];
                    const double2 h21 = H[cur][q1][p2], h22 = H[cur][q1][q2];
                    const double2 s11 = S[cur][p1][p2], s12 = S[cur][p1][q2];
                    const double2 s21 = S[cur][q1][p2], s22 = S[cur][q1][q2];
                    if (!ar && !ac) {
                        H[nxt][p1][p2] = h11;
                        H[nxt][p1][q2] = h12;
                        H[nxt][q1][p2] = h21;
                        H[nxt][q1][q2] = h22;
                        S[nxt][p1][p2] = s11;
                        S[nxt][p1][q2] = s12;
                        S[nxt][q1][p2] = s21;
                        S[nxt][q1][q2] = s22;
                    } else {
                        double2 r11 = one, r21 = zero, r12 = zero, r22 = one;
                        if (ar) {
                            r11 = now.z[kr][0];
                            r21 = now.z[kr][1];
                            r12 = now.z[kr][2];
                            r22 = now.z[kr][3];
                        }
                        double2 x11 = mac2(h11, c11, h12, c21), x12 = mac2(h11, c12, h12, c22);
                        double2 x21 = mac2(h21, c11, h22, c21), x22 = mac2(h21, c12, h22, c22);
                        H[nxt][p1][p2] = macc2(r11, x11, r21, x21);
                        H[nxt][p1][q2] = macc2(r11, x12, r21, x22);
                        H[nxt][q1][p2] = macc2(r12, x11, r22, x21);
                        H[nxt][q1][q2] = macc2(r12, x12, r22, x22);
                        x11 = mac2(s11, c11, s12, c21);
                        x12 = mac2(s11, c12, s12, c22);
                        x21 = mac2(s21, c11, s22, c21);
                        x22 = mac2(s21, c12, s22, c22);
                        S[nxt][p1][p2] = macc2(r11, x11, r21, x21);
                        S[nxt][p1][q2] = macc2(r11, x12, r21, x22);
                        S[nxt][q1][p2] = macc2(r12, x11, r22, x21);
                        S[nxt][q1][q2] = macc2(r12, x12, r22, x22);
                    }
                } else if (ac) {
                    const double2 w11 = Zs[p1][p2], w12 = Zs[p1][q2];
                    const double2 w21 = Zs[q1][p2], w22 = Zs[q1][q2];
                    Zs[p1][p2] = mac2(w11, c11, w12, c21);
                    Zs[p1][q2] = mac2(w11, c12, w12, c22);
                    Zs[q1][p2] = mac2(w21, c11, w22, c21);
                    Zs[q1][q2] = mac2(w21, c12, w22, c22);
                }
            }
        }
        __syncthreads();
    }
        if (isw + 1 >= max_isw || !more[isw & 1]) break;
    }
    const GPtr<double2> Z64(A.zh64 + (size_t)bpi * PB * PB);
    const GPtr<float2> Z32(F32 ? A.zh32 + (size_t)bpi * PB * PB : A.zh32);
    for (int idx = tid; idx < PB * PB; idx += inner_threads<PB>()) {
        const int i = idx % PB, j = idx / PB;
        const double2 z = Zs[i][j];
        Z64.st(idx, z);
        if (F32) Z32.st(idx, make_float2((float)z.x, (float)z.y));
    }
    if (tid < kWave) {
        cv = wave_sum(cv);
        ct = wave_sum(ct);
        cbig = wave_sum(cbig);
        if (tid == 0) {
            GPtr<int>(A.ntr).st(bpi, (int)ct);
            const GPtr<unsigned long long> cn = GPtr<unsigned long long>(A.bcnt) + 3 * bpi;
            cn.st(0, cn.ld(0) + (unsigned long long)cv);
            cn.st(1, cn.ld(1) + (unsigned long long)ct);
            cn.st(2, cn.ld(2) + (unsigned long long)cbig);
        }
    }
}

// Inner sweep for 64 pivot columns.  (H^, S^) are kept in LDS as packed
// upper triangles, single-buffered and updated in place; Z^ is a full 64 x 64
// LDS array (column-major).  An inner step runs in two phases separated by a
// barrier: every thread first reads what the step needs (the pivot
// wavefront its look-ahead operands for the next step, each block thread its
// 2x2 blocks), then the block threads write their updated blocks while the
// pivot wavefront computes the next step's 2x2 steps and the Z^ threads
// update Z^.  Threads: the pivot wavefront (lanes 0-31 form the (p,p) and
// (p,q) entries of pair k = lane and run its 2x2 step, lanes 32-63 form the
// (q,q) entries), one thread per unordered pair of pair slots {kr <= kc}
// (528; it forms Z_kr^* M Z_kc and stores the entries on or above the
// diagonal, conjugated where the block lies below it), and 432 threads for
// row segments of Z^ (row i, slot k), which also build the next-but-one
// step's look-ahead table.  The look-ahead forms each entry in the
// orientation of the thread that stores it (rows from the smaller slot,
// conjugated after), so the two agree bit for bit.
constexpr int kI64Threads = 1024;
constexpr int kI64Blocks = 32 * 33 / 2;
constexpr int kI64ZThreads = kI64Threads - kWave - kI64Blocks;

__device__ __forceinline__ double2 hget(const double2 *M, int i, int j) {
    return i <= j ? M[pk_idx(i, j)] : cconj(M[pk_idx(j, i)]);
}

// Look-ahead operands of entry kind e ((p,p), (q,q), (p,q)) of pair slot k
// at inner step is following step prev, packed as for lookahead_entry; bit
// 1 of the byte of ii marks an entry formed transposed and conjugated after.
__device__ __forceinline__ uint2 lookahead64(const InnerOrder &ord, int is, int prev, int k, int e,
                                             int c) {
    int pp = -1, qq = -1;
    if (k < ord.slots()) ord.pair(is, k, pp, qq);
    if (!(k < ord.slots() && qq < c)) return make_uint2(0u, kNoEntry);
    int i = (e == 1) ? qq : pp, j = (e == 0) ? pp : qq;
    int ki, ii, kj, jj;
    ord.where(prev, i, ki, ii);
    ord.where(prev, j, kj, jj);
    int cj = 0;
    if (ki > kj) {
        int t = ki;
        ki = kj;
        kj = t;
        t = ii;
        ii = jj;
        jj = t;
        cj = 1;
    }
    int r0, r1, c0, c1;
    ord.pair(prev, ki, r0, r1);
    ord.pair(prev, kj, c0, c1);
    return make_uint2((unsigned)r0 | (unsigned)r1 << 8 | (unsigned)c0 << 16 | (unsigned)c1 << 24,
                      (unsigned)ki | (unsigned)(ii | cj << 1) << 8 | (unsigned)kj << 16 |
                          (unsigned)jj << 24);
}

// One look-ahead entry: r^* M c over the 2x2 block of the previous step
// (same expressions as the block update), from the packed matrix.
__device__ __forceinline__ double2 lookahead_value(const double2 *M, uint2 te,
                                                   const InnerStep<64> &prev) {
    const double2 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0);
    const int r0 = te.x & 0xff, r1 = (te.x >> 8) & 0xff;
    const int c0 = (te.x >> 16) & 0xff, c1 = te.x >> 24;
    const int ki = te.y & 0xff, iib = (te.y >> 8) & 0xff;
    const int kj = (te.y >> 16) & 0xff, jj = te.y >> 24;
    const int ii = iib & 1;
    const int ai = prev.act[ki], aj = prev.act[kj];
    const double2 za = prev.z[ki][2 * ii], zb = prev.z[ki][2 * ii + 1];
    const double2 zc = prev.z[kj][2 * jj], zd = prev.z[kj][2 * jj + 1];
    const double2 h00 = hget(M, r0, c0), h01 = hget(M, r0, c1);
    const double2 h10 = hget(M, r1, c0), h11 = hget(M, r1, c1);
    const double2 ra = ai ? za : (ii ? zero : one), rb = ai ? zb : (ii ? one : zero);
    const double2 ca = aj ? zc : (jj ? zero : one), cb = aj ? zd : (jj ? one : zero);
    const double2 v = macc2(ra, mac2(h00, ca, h01, cb), rb, mac2(h10, ca, h11, cb));
    return (iib & 2) ? cconj(v) : v;
}

template <int F32, int FB>
__global__ __launch_bounds__(kI64Threads) void k_blk_inner64(const PencilDev *PD, const int *pre,
                                                            const int *flag, int B, int crit,
                                                            int step, int cross_mode) {
    constexpr int PB = 64, NP = 32;
    constexpr int max_isw = FB ? kFbSweeps : 1;  // FB: inner sweeps as in k_blk_inner
    __shared__ double2 H[kG64Packed];
    __shared__ double2 S[kG64Packed];
    __shared__ double2 Zs[PB][PB + 1];  // Zs[column][row]
    __shared__ InnerStep<PB> st[2];
    __shared__ uint2 tab[2][3 * NP];     // look-ahead operands, by the parity of the step
    __shared__ int more[2];              // FB: another inner sweep follows (by parity)
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int bpi = pencil_local(pre, pk, blockIdx.x);
    const int tid = threadIdx.x;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) {
        if (tid == 0) GPtr<int>(A.ntr).st(bpi, 0);
        return;
    }
    if (tid < kWave) __builtin_amdgcn_s_setprio(3);
    InnerOrder ord;
    ord.cross = !FB && cross_mode == GHSVD_INNER_CROSS && step > 0 && ca == NP && cb == NP;
    ord.C = c + (c & 1);
    ord.w = NP;
    const int nsteps = ord.steps(), nsl = ord.slots();
    // this thread's block slots (block threads) or Z^ lane (Z^ threads)
    const int tb = tid - kWave, tz = tb - kI64Blocks;
    int kr = 0, kc = 0;
    if (tb >= 0 && tb < kI64Blocks) {
        kc = (int)((sqrtf(8.0f * (float)tb + 1.0f) - 1.0f) * 0.5f);
        while ((kc + 1) * (kc + 2) / 2 <= tb) ++kc;
        while (kc * (kc + 1) / 2 > tb) --kc;
        kr = tb - kc * (kc + 1) / 2;
    }
    {
        const GPtr<double2> G(A.gp + (size_t)bpi * 2 * kG64Packed);
        for (int idx = tid; idx < kG64Packed; idx += kI64Threads) {
            H[idx] = G.ld(idx);
            S[idx] = G.ld(kG64Packed + idx);
        }
        for (int idx = tid; idx < PB * PB; idx += kI64Threads) {
            const int col = idx / PB, row = idx % PB;
            Zs[col][row] = cmk(row == col ? 1.0 : 0.0, 0.0);
        }
        if (tid < 3 * NP) {
            if (nsteps > 1) tab[1][tid] = lookahead64(ord, 1, 0, tid % NP, tid / NP, c);
            else if (FB) tab[1][tid] = lookahead64(ord, 0, 0, tid % NP, tid / NP, c);
        }
    }
    __syncthreads();
    const double tol = (F32 ? 0x1p-23 : 0x1p-52) * sqrt((double)c);
    double cv = 0.0, ct = 0.0, cbig = 0.0;
    // the 2x2 steps of inner step 0 from the entries as stored
    if (tid < NP) {
        const int k = tid;
        int pp = -1, qq = -1;
        if (k < nsl) ord.pair(0, k, pp, qq);
        int kind = kSkip;
        if (k < nsl && qq < c) {
            const double2 hpq = hget(H, pp, qq), spq = hget(S, pp, qq);
            Zp z;
            kind = hz_step_fast(H[pk_idx(pp, pp)].x, H[pk_idx(qq, qq)].x, hpq, S[pk_idx(pp, pp)].x,
                                S[pk_idx(qq, qq)].x, spq, tol, crit, z, F32);
            cv += 1.0;
            if (kind == GHSVD_ENONFINITE) atomicCAS(&A.st->err, 0, GHSVD_ENONFINITE);
            if (kind < 0) kind = kSkip;
            st[0].z[k][0] = z.z11;
            st[0].z[k][1] = z.z21;
            st[0].z[k][2] = z.z12;
            st[0].z[k][3] = z.z22;
            ct += kind > 0 ? 1.0 : 0.0;
            cbig += kind == kBig ? 1.0 : 0.0;
        }
        st[0].act[k] = kind > 0;
    }
    __syncthreads();
    double cmark = 0.0;  // ct at the end of the previous inner sweep
    int g = 0;           // inner steps so far (parity of the step and table buffers)
    for (int isw = 0;; ++isw) {
    for (int s = 0; s < nsteps; ++s, ++g) {
        const int cur = g & 1, nxt = cur ^ 1;
        const InnerStep<PB> &now = st[cur];
        // ---- phase 1: reads ----
        double2 hv0 = cmk(0.0, 0.0), sv0 = hv0, hv2 = hv0, sv2 = hv0;
        bool mine0 = false, mine2 = false;
        double2 bh[4], bs[4];
        int p1 = 0, q1 = 0, p2 = 0, q2 = 0;
        bool blk = false;
        bool go = false;  // pivot wavefront: a next inner step follows
        if (tid < kWave) {
            go = s + 1 < nsteps;
            if (!go && isw + 1 < max_isw) {
                // the pivots of this sweep's last step are in ct: another
                // sweep follows when the sweep applied any transformation
                const double sa = wave_sum(ct - cmark);
                cmark = ct;
                go = sa > 0.0;
                if (tid == 0) more[isw & 1] = go;
            }
            if (go) {
                const uint2 te0 = tab[nxt][tid];  // (p,p) for lanes < 32, (q,q) above
                mine0 = te0.y != kNoEntry;
                if (mine0) {
                    hv0 = lookahead_value(H, te0, now);
                    sv0 = lookahead_value(S, te0, now);
                }
                if (tid < NP) {
                    const uint2 te2 = tab[nxt][2 * NP + tid];  // (p,q)
                    mine2 = te2.y != kNoEntry;
                    if (mine2) {
                        hv2 = lookahead_value(H, te2, now);
                        sv2 = lookahead_value(S, te2, now);
                    }
                }
            }
        } else if (tb < kI64Blocks) {
            blk = kr < nsl && kc < nsl && (now.act[kr] || now.act[kc]);
            if (blk) {
                ord.pair(s, kr, p1, q1);
                ord.pair(s, kc, p2, q2);
                bh[0] = hget(H, p1, p2);
                bh[1] = hget(H, p1, q2);
                bh[2] = hget(H, q1, p2);
                bh[3] = hget(H, q1, q2);
                bs[0] = hget(S, p1, p2);
                bs[1] = hget(S, p1, q2);
                bs[2] = hget(S, q1, p2);
                bs[3] = hget(S, q1, q2);
            }
        }
        __syncthreads();
        // ---- phase 2: writes ----
        if (tid < kWave) {
            if (go) {
                // gather (q,q) of pair k from lane k + 32 (every lane takes part)
                const double hqq = lane_plus32(hv0.x), sqq = lane_plus32(sv0.x);
                if (tid < NP) {
                    const int k = tid;
                    int kind = kSkip;
                    if (mine0 && mine2) {
                        Zp z;
                        kind = hz_step_fast(hv0.x, hqq, hv2, sv0.x, sqq, sv2, tol, crit, z, F32);
                        cv += 1.0;
                        if (kind == GHSVD_ENONFINITE) atomicCAS(&A.st->err, 0, GHSVD_ENONFINITE);
                        if (kind < 0) kind = kSkip;
                        st[nxt].z[k][0] = z.z11;
                        st[nxt].z[k][1] = z.z21;
                        st[nxt].z[k][2] = z.z12;
                        st[nxt].z[k][3] = z.z22;
                        ct += kind > 0 ? 1.0 : 0.0;
                        cbig += kind == kBig ? 1.0 : 0.0;
                    }
                    st[nxt].act[k] = kind > 0;
                }
            }
        } else if (tb < kI64Blocks) {
            if (blk) {
                const double2 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0);
                const bool ar = now.act[kr], ac = now.act[kc];
                double2 r11 = one, r21 = zero, r12 = zero, r22 = one;
                double2 c11 = one, c21 = zero, c12 = zero, c22 = one;
                if (ar) {
                    r11 = now.z[kr][0];
                    r21 = now.z[kr][1];
                    r12 = now.z[kr][2];
                    r22 = now.z[kr][3];
                }
                if (ac) {
                    c11 = now.z[kc][0];
                    c21 = now.z[kc][1];
                    c12 = now.z[kc][2];
                    c22 = now.z[kc][3];
                }
                double2 *M = H;
                double2 *m = bh;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const double2 x11 = mac2(m[0], c11, m[1], c21), x12 = mac2(m[0], c12, m[1], c22);
                    const double2 x21 = mac2(m[2], c11, m[3], c21), x22 = mac2(m[2], c12, m[3], c22);
                    const double2 n11 = macc2(r11, x11, r21, x21), n12 = macc2(r11, x12, r21, x22);
                    const double2 n21 = macc2(r12, x11, r22, x21), n22 = macc2(r12, x12, r22, x22);
                    if (kr == kc) {
                        // the diagonal block: (p,p), (q,q) and one of (p,q), (q,p)
                        M[pk_idx(p1, p1)] = n11;
                        M[pk_idx(q1, q1)] = n22;
                        if (p1 < q1) M[pk_idx(p1, q1)] = n12;
                        else M[pk_idx(q1, p1)] = n21;
                    } else {
                        if (p1 <= p2) M[pk_idx(p1, p2)] = n11; else M[pk_idx(p2, p1)] = cconj(n11);
                        if (p1 <= q2) M[pk_idx(p1, q2)] = n12; else M[pk_idx(q2, p1)] = cconj(n12);
                        if (q1 <= p2) M[pk_idx(q1, p2)] = n21; else M[pk_idx(p2, q1)] = cconj(n21);
                        if (q1 <= q2) M[pk_idx(q1, q2)] = n22; else M[pk_idx(q2, q1)] = cconj(n22);
                    }
                    M = S;
                    m = bs;
                }
            }
        } else {
            // Z^ <- Z^ Z_k on the columns of each active slot k, row by row
            for (int u = tz; u < PB * NP; u += kI64ZThreads) {
                const int row = u % PB, k = u / PB;
                if (k < nsl && now.act[k]) {
                    int pp, qq;
                    ord.pair(s, k, pp, qq);
                    const double2 c11 = now.z[k][0], c21 = now.z[k][1];
                    const double2 c12 = now.z[k][2], c22 = now.z[k][3];
                    const double2 w1 = Zs[pp][row], w2 = Zs[qq][row];
                    Zs[pp][row] = mac2(w1, c11, w2, c21);
                    Zs[qq][row] = mac2(w1, c12, w2, c22);
                }
            }
            // operands of the step after next (in FB, across the end of a sweep)
            if ((FB || s + 2 < nsteps) && tz < 3 * NP) {
                const int t2 = (s + 2) % nsteps, t1 = (s + 1) % nsteps;
                tab[cur][tz] = lookahead64(ord, t2, t1, tz % NP, tz / NP, c);
            }
        }
        __syncthreads();
    }
        if (isw + 1 >= max_isw || !more[isw & 1]) break;
    }
    const GPtr<double2> Z64(A.zh64 + (size_t)bpi * PB * PB);
    const GPtr<float2> Z32(F32 ? A.zh32 + (size_t)bpi * PB * PB : A.zh32);
    for (int idx = tid; idx < PB * PB; idx += kI64Threads) {
        const int i = idx % PB, j = idx / PB;
        const double2 z = Zs[j][i];
        Z64.st(idx, z);
        if (F32) Z32.st(idx, make_float2((float)z.x, (float)z.y));
    }
    if (tid < kWave) {
        cv = wave_sum(cv);
        ct = wave_sum(ct);
        cbig = wave_sum(cbig);
        if (tid == 0) {
            GPtr<int>(A.ntr).st(bpi, (int)ct);
            const GPtr<unsigned long long> cn = GPtr<unsigned long long>(A.bcnt) + 3 * bpi;
            cn.st(0, cn.ld(0) + (unsigned long long)cv);
            cn.st(1, cn.ld(1) + (unsigned long long)ct);
            cn.st(2, cn.ld(2) + (unsigned long long)cbig);
        }
    }
}

// F_C <- F_C Z^, G_C <- G_C Z^, Z_C <- Z_C Z^ for one block pair, in place
// (Section 6.4.3), skipped when the inner sweep applied no transformation.
// The rows of F, G and Z form 16-row strips (tf + tg + tz of them); a
// workgroup's four wavefronts take kUpdStrips strips each, interleaved, and
// load the next strip while the matrix cores work on the current one.  A
// wavefront forms the strip's transpose, D = Z^T X^T, with the 16x16x4
// MFMA: lane j + 16 k loads row j of pivot column k (the B operand; 16
// lanes read 16 consecutive rows of one column), the A operands Z^[k][i]
// are read once straight into registers, and lane l holds
// D[i][l % 16] = (X Z^)[l % 16][i], so 16
// lanes store 256 contiguous bytes of one column.  Every read of a strip
// precedes its writes within the wavefront, and strips are disjoint.
constexpr int kUpdStrips = 6;
// Strips per wavefront of the update: the 64-column form does four times the
// products per strip, and takes fewer strips so that a 1024-column pencil
// still spreads over every CU.
__host__ __device__ constexpr int upd_strips(int w) { return w == 32 ? 3 : kUpdStrips; }

// Matrix, leading dimension and row of lane row j of strip st (F, G, Z
// strips in that order); ok = 0 past the last row or the last strip.
template <typename C2>
__device__ __forceinline__ GPtr<C2> strip_of(const PencilDev &A, int st, int j, long &ld, int &row,
                                            bool &ok) {
    constexpr bool F32 = sizeof(C2) == 8;
    C2 *X;
    int rows;
    if (st < A.tf) {
        X = reinterpret_cast<C2 *>(F32 ? (void *)A.F32 : (void *)A.Fw);
        ld = A.ldf;
        rows = A.mr;
    } else if (st < A.tf + A.tg) {
        st -= A.tf;
        X = reinterpret_cast<C2 *>(F32 ? (void *)A.G32 : (void *)A.Gw);
        ld = A.ldg;
        rows = A.pr;
    } else {
        st -= A.tf + A.tg;
        X = reinterpret_cast<C2 *>(F32 ? (void *)A.Z32 : (void *)A.Zw);
        ld = A.ldz;
        rows = A.n;
    }
    row = st * 16 + j;
    ok = row < rows && st < (A.tf + A.tg + A.tz);
    if (!ok) row = rows - 1;  // an in-bounds address for the unconditional load
    return GPtr<C2>(X);
}

template <typename T, int PB>
__global__ __launch_bounds__(256) void k_blk_update(const PencilDev *PD, const int *pre,
                                                    const int *flag, int B, int step) {
    using C2 = typename Mfma<T>::c2;
    using ACC = typename Mfma<T>::acc;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NTD = PB / 16;  // output column tiles
    constexpr int KS = PB / 4;    // k-steps
    constexpr int NS = upd_strips(PB / 2);  // strips per wavefront
    // 32 and 64 columns: Z^ is staged in LDS (in registers it would hold 64
    // VGPRs of the 32-column kernel for all strips and cut its occupancy to
    // two wavefronts per SIMD)
    constexpr bool ZL = PB >= 32;
    __shared__ C2 Zl[ZL ? PB : 1][ZL ? PB + 1 : 1];
    const int pk = find_pencil(pre, B, blockIdx.x);
    const PencilDev A = PD[pk];
    if (step >= A.nb - 1 || flag[pk]) return;
    const int local = pencil_local(pre, pk, blockIdx.x);
    const int bpi = local / A.tu, g = local % A.tu;
    if (GPtr<int>(A.ntr).ld(bpi) == 0) return;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int nstrips = A.tf + A.tg + A.tz;
    // this lane's global columns of the B operand (pivot column 4 ks + kq)
    long cofs[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int cc = 4 * ks + kq;
        cofs[ks] = cc < c ? (long)blk_col(A.w, a, b, ca, cc) : -1;
    }
    // the A operands Z^[4 ks + kq][16 ti + j] (Z^ column-major, PB x PB):
    // staged once in LDS (32 and 64 columns), or read straight into
    // registers, where they stay for all strips (16 columns)
    C2 za[ZL ? 1 : KS][NTD];
    if constexpr (ZL) {
        for (int idx = tid; idx < PB * PB; idx += 256) {
            const long e = (long)bpi * PB * PB + idx;
            if constexpr (F32) {
                Zl[idx % PB][idx / PB] = GPtr<float2>(A.zh32).ld(e);
            } else {
                Zl[idx % PB][idx / PB] = GPtr<double2>(A.zh64).ld(e);
            }
        }
        __syncthreads();
    } else {
        const long zb = (long)bpi * PB * PB;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int ti = 0; ti < NTD; ++ti) {
                const long e = zb + (4 * ks + kq) + (long)PB * (ti * 16 + j);
                if constexpr (F32) {
                    za[ks][ti] = GPtr<float2>(A.zh32).ld(e);
                } else {
                    za[ks][ti] = GPtr<double2>(A.zh64).ld(e);
                }
            }
    }
    C2 xb[KS], xn[KS];
    const int st0 = g * NS * 4 + wv;
    {
        long ld;
        int row;
        bool ok;
        const GPtr<C2> X = strip_of<C2>(A, st0 < nstrips ? st0 : 0, j, ld, row, ok);
        ok = ok && st0 < nstrips;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const T msk = (ok && cofs[ks] >= 0) ? T(1) : T(0);
            C2 v = X.ld((cofs[ks] >= 0 ? cofs[ks] : 0L) * ld + row);
            v.x *= msk;
            v.y *= msk;
            xb[ks] = v;
        }
    }
#pragma unroll
    for (int it = 0; it < NS; ++it) {
        const int st = st0 + 4 * it;
        if (it + 1 < NS) {
            long ld;
            int row;
            bool ok;
            const int sn = st + 4;
            const GPtr<C2> X = strip_of<C2>(A, sn < nstrips ? sn : 0, j, ld, row, ok);
            ok = ok && sn < nstrips;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const T msk = (ok && cofs[ks] >= 0) ? T(1) : T(0);
                C2 v = X.ld((cofs[ks] >= 0 ? cofs[ks] : 0L) * ld + row);
                v.x *= msk;
                v.y *= msk;
                xn[ks] = v;
            }
        }
        ACC acc_re[NTD], acc_im[NTD];
#pragma unroll
        for (int ti = 0; ti < NTD; ++ti) {
            acc_re[ti] = ACC{0, 0, 0, 0};
            acc_im[ti] = ACC{0, 0, 0, 0};
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int ti = 0; ti < NTD; ++ti) {
                C2 z;
                if constexpr (ZL) {
                    z = Zl[4 * ks + kq][ti * 16 + j];
                } else {
                    z = za[ks][ti];
                }
                // (X Z^) = X_re Z_re - X_im Z_im + i (X_re Z_im + X_im Z_re)
                acc_re[ti] = Mfma<T>::mma(z.x, xb[ks].x, acc_re[ti]);
                acc_re[ti] = Mfma<T>::mma(-z.y, xb[ks].y, acc_re[ti]);
                acc_im[ti] = Mfma<T>::mma(z.y, xb[ks].x, acc_im[ti]);
                acc_im[ti] = Mfma<T>::mma(z.x, xb[ks].y, acc_im[ti]);
            }
        if (st < nstrips) {
            long ld;
            int row;
            bool ok;
            const GPtr<C2> X = strip_of<C2>(A, st, j, ld, row, ok);
            if (ok) {
#pragma unroll
                for (int ti = 0; ti < NTD; ++ti)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int oc = ti * 16 + Mfma<T>::row(lane, r);
                        if (oc < c) {
                            C2 v;
                            v.x = acc_re[ti][r];
                            v.y = acc_im[ti][r];
                            X.st((long)blk_col(A.w, a, b, ca, oc) * ld + row, v);
                        }
                    }
            }
        }
        if (it + 1 < NS) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) xb[ks] = xn[ks];
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 stage helpers: conversions and the FP64 hand-off GEMM C = A B, with A
// complex128 (rows x n), B complex64 (n x n), C complex128 (MFMA FP64).
// ---------------------------------------------------------------------------
__global__ void k_to_f32(int rows, int n, const double2 *src, long lds, float2 *dst, long ldd) {
    const int j = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        const double2 v = src[(size_t)j * lds + r];
        dst[(size_t)j * ldd + r] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_to_f64(int rows, int n, const float2 *src, long lds, double2 *dst, long ldd) {
    const int j = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        const float2 v = src[(size_t)j * lds + r];
        dst[(size_t)j * ldd + r] = make_double2((double)v.x, (double)v.y);
    }
}

constexpr int kGemmT = 64;  // output tile (rows and columns)
constexpr int kGemmK = 16;  // k chunk staged in LDS

__global__ __launch_bounds__(256) void k_handoff_gemm(int rows, int n, const double2 *Am, long lda,
                                                      const float2 *Bm, long ldb, double2 *Cm,
                                                      long ldc) {
    __shared__ double2 As[kGemmT][kGemmK + 1];  // [row][k]
    __shared__ double2 Bs[kGemmK][kGemmT + 1];  // [k][col]
    const int r0 = blockIdx.x * kGemmT, c0 = blockIdx.y * kGemmT;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wi = wv & 1, wj = wv >> 1;  // 2 x 2 waves, 32 x 32 each
    v4d acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc_re[a][b] = v4d{0, 0, 0, 0};
            acc_im[a][b] = v4d{0, 0, 0, 0};
        }
    for (int k0 = 0; k0 < n; k0 += kGemmK) {
        for (int idx = tid; idx < kGemmT * kGemmK; idx += 256) {
            const int rr = idx % kGemmT, kk = idx / kGemmT;
            double2 v = cmk(0.0, 0.0);
            if (r0 + rr < rows && k0 + kk < n) v = Am[(size_t)(k0 + kk) * lda + r0 + rr];
            As[rr][kk] = v;
        }
        for (int idx = tid; idx < kGemmK * kGemmT; idx += 256) {
            const int kk = idx % kGemmK, cc = idx / kGemmK;
            double2 v = cmk(0.0, 0.0);
            if (k0 + kk < n && c0 + cc < n) {
                const float2 f = Bm[(size_t)(c0 + cc) * ldb + k0 + kk];
                v = cmk((double)f.x, (double)f.y);
            }
            Bs[kk][cc] = v;
        }
        __syncthreads();
        for (int kq = 0; kq < kGemmK; kq += 4) {
            const int k = kq + (lane >> 4);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double2 x = As[wi * 32 + a * 16 + (lane & 15)][k];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double2 y = Bs[k][wj * 32 + b * 16 + (lane & 15)];
                    acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, acc_re[a][b], 0, 0, 0);
                    acc_re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.y, y.y, acc_re[a][b], 0, 0, 0);
                    acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.y, acc_im[a][b], 0, 0, 0);
                    acc_im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.x, acc_im[a][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wi * 32 + a * 16 + Mfma<double>::row(lane, r);
                const int col = c0 + wj * 32 + b * 16 + (lane & 15);
                if (row < rows && col < n) Cm[(size_t)col * ldc + row] = cmk(acc_re[a][b][r], acc_im[a][b][r]);
            }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
void set_block_geometry(PencilDev &d, int w) {
    d.w = w;
    d.nb = (d.n + w - 1) / w;
    if (d.nb & 1) d.nb += 1;
    d.nbp = d.nb / 2;
    const int chunk = w == 32 ? kG64Chunk : kGramChunk;
    d.kf = (d.mr + chunk - 1) / chunk;
    d.kg = (d.pr + chunk - 1) / chunk;
    d.tf = (d.mr + 15) / 16;
    d.tg = (d.pr + 15) / 16;
    d.tz = (d.n + 15) / 16;
    d.tu = (d.tf + d.tg + d.tz + 4 * upd_strips(w) - 1) / (4 * upd_strips(w));
}

int pick_block_width(int max_n, int requested) {
    if (requested == 8 || requested == 16 || requested == 32) return requested;
    return max_n >= 512 ? 16 : 8;
}

void carve_blocked(Carver &c, int mr, int n, int pr, int w, int mixed, PencilDev &d) {
    PencilDev g{};
    g.mr = mr;
    g.n = n;
    g.pr = pr;
    set_block_geometry(g, w);
    const size_t pb2 = (size_t)(2 * w) * (2 * w);
    d.part = c.take<double2>((size_t)g.nbp * (g.kf + g.kg) * pb2);
    d.zh64 = c.take<double2>((size_t)g.nbp * pb2);
    d.zh32 = c.take<float2>((size_t)g.nbp * pb2);
    d.gp = w == 32 ? c.take<double2>((size_t)g.nbp * 2 * kG64Packed) : nullptr;
    d.ntr = c.take<int>(g.nbp);
    d.bcnt = c.take<unsigned long long>(3 * (size_t)g.nbp);
    if (mixed) {
        const long ld = pad_ld(mr > pr ? mr : pr);
        d.tmp = c.take<double2>((size_t)ld * n);
    }
}

size_t blocked_bytes(int mr, int n, int pr, int w, int mixed) {
    Carver c{nullptr, 0, (size_t)-1};
    PencilDev d{};
    carve_blocked(c, mr, n, pr, w, mixed, d);
    return c.used + 256;
}

using BlkInnerFn = void (*)(const PencilDev *, const int *, const int *, int, int, int, int);

struct BlockedArg {
    BlkFn gram, gsum, upd;  // gsum: chunk sums of the 64-column Grams (else null)
    BlkInnerFn inner;
    int inner_nt;
    int crit;
    int mode;  // inner_order
    int fp32;  // FP32 warm-up kernels (timed under their own kinds)
};

static int blocked_step(const BatchCtx &c, const void *arg, int step, hipStream_t s) {
    const BlockedArg *a = static_cast<const BlockedArg *>(arg);
    // kernel timing events are taken unless the batch is plain (no events)
    const bool tm = !c.plain;
    const int kg = a->fp32 ? kProfGram32 : kProfGram, ki = a->fp32 ? kProfInner32 : kProfInner,
              ku = a->fp32 ? kProfUpdate32 : kProfUpdate;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) prof_take(kg, e0, e1);
    const dim3 gb(a->gsum ? kWave * kG64Tiles : kWave * kGramWaves);
    if (a->gsum) {
        launch_ev(a->gram, dim3(c.total(BatchCtx::kGram)), gb, 0, s, e0, nullptr, c.dev,
                  c.pre_of(BatchCtx::kGram), c.flag_dev, c.B, step);
        launch_ev(a->gsum, dim3(c.total(BatchCtx::kBp), 2 * kG64Tiles), dim3(256), 0, s, nullptr,
                  e1, c.dev, c.pre_of(BatchCtx::kBp), c.flag_dev, c.B, step);
    } else {
        launch_ev(a->gram, dim3(c.total(BatchCtx::kGram)), gb, 0, s, e0, e1, c.dev,
                  c.pre_of(BatchCtx::kGram), c.flag_dev, c.B, step);
    }
    prof_done(kg, e0, e1);
    e0 = e1 = nullptr;
    if (tm) prof_take(ki, e0, e1);
    launch_ev(a->inner, dim3(c.total(BatchCtx::kBp)), dim3(a->inner_nt), 0, s, e0, e1, c.dev,
              c.pre_of(BatchCtx::kBp), c.flag_dev, c.B, a->crit, step, a->mode);
    prof_done(ki, e0, e1);
    e0 = e1 = nullptr;
    if (tm) prof_take(ku, e0, e1);
    launch_ev(a->upd, dim3(c.total(BatchCtx::kUpd)), dim3(256), 0, s, e0, e1, c.dev,
              c.pre_of(BatchCtx::kUpd), c.flag_dev, c.B, step);
    prof_done(ku, e0, e1);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

BlkFn block_update_kernel(int w) {
    if (w == 32) return k_blk_update<double, 64>;
    if (w == 16) return k_blk_update<double, 32>;
    if (w == 8) return k_blk_update<double, 16>;
    return nullptr;
}

int run_blocked_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, int inner_order,
                      hipStream_t s, std::vector<SweepResult> &res,
                      const std::vector<int> *presolved) {
    if (inner_shortened(inner_order)) {
        // (J)QR-shortened block pivots in the FP64 stage; the FP32 warm-up
        // forms them as Grams with the same inner ordering
        const bool fbo = inner_order == GHSVD_INNER_FB_JQR || inner_order == GHSVD_INNER_ML_FB;
        if (!fp32)
            return run_blocked_shortened(c, max_sweeps, crit, fbo, inner_multilevel(inner_order),
                                         s, res);
        inner_order = fbo ? GHSVD_INNER_FB : GHSVD_INNER_FULL;
    }
    int w = 0, steps = 1;
    for (const PencilDev &P : c.host) {
        if (w == 0) w = P.w;
        if (P.w != w) return GHSVD_EINVAL;  // one block width per batch
        if (P.nb - 1 > steps) steps = P.nb - 1;
    }
    if (c.total(BatchCtx::kBp) == 0) {
        res.assign(c.B, SweepResult{GHSVD_OK, 0, 1, 0, 0, 0});
        return GHSVD_OK;
    }
    BlockedArg a{};
    a.crit = crit;
    a.mode = inner_order;
    a.fp32 = fp32;
    const bool fb = inner_order == GHSVD_INNER_FB;
    if (w == 32) {
        a.gram = fp32 ? k_blk_gram64<float> : k_blk_gram64<double>;
        a.gsum = fp32 ? k_blk_gsum64<float> : k_blk_gsum64<double>;
        a.inner = fb ? (fp32 ? k_blk_inner64<1, 1> : k_blk_inner64<0, 1>)
                     : (fp32 ? k_blk_inner64<1, 0> : k_blk_inner64<0, 0>);
        a.inner_nt = kI64Threads;
        a.upd = fp32 ? k_blk_update<float, 64> : k_blk_update<double, 64>;
    } else if (w == 16) {
        a.gram = fp32 ? k_blk_gram<float, 32> : k_blk_gram<double, 32>;
        a.inner = fb ? (fp32 ? k_blk_inner<32, 1, 1> : k_blk_inner<32, 0, 1>)
                     : (fp32 ? k_blk_inner<32, 1, 0> : k_blk_inner<32, 0, 0>);
        a.inner_nt = inner_threads<32>();
        a.upd = fp32 ? k_blk_update<float, 32> : k_blk_update<double, 32>;
    } else if (w == 8) {
        a.gram = fp32 ? k_blk_gram<float, 16> : k_blk_gram<double, 16>;
        a.inner = fb ? (fp32 ? k_blk_inner<16, 1, 1> : k_blk_inner<16, 0, 1>)
                     : (fp32 ? k_blk_inner<16, 1, 0> : k_blk_inner<16, 0, 0>);
        a.inner_nt = inner_threads<16>();
        a.upd = fp32 ? k_blk_update<float, 16> : k_blk_update<double, 16>;
    } else {
        return GHSVD_EINVAL;
    }
    return drive_stage(c, max_sweeps, fp32, 1, blocked_step, &a, steps,
                       fp32 ? "blocked-fp32" : "blocked-fp64", s, res, presolved);
}

int to_fp32(const BatchCtx &c, hipStream_t s) {
    for (const PencilDev &P : c.host) {
        const int n = P.n;
        int bx = (P.mr + 255) / 256;
        if (bx > 16) bx = 16;
        hipLaunchKernelGGL(k_to_f32, dim3(bx, n), dim3(256), 0, s, P.mr, n, P.Fw, P.ldf, P.F32, P.ldf);
        bx = (P.pr + 255) / 256;
        if (bx > 16) bx = 16;
        hipLaunchKernelGGL(k_to_f32, dim3(bx, n), dim3(256), 0, s, P.pr, n, P.Gw, P.ldg, P.G32, P.ldg);
        int rc = set_identity(n, P.Z32, P.ldz, 1, s);
        if (rc) return rc;
    }
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// Hand-off after the FP32 stage: F <- F Z32, G <- G Z32 in FP64, Z <- Z32.
int fp32_handoff(const BatchCtx &c, hipStream_t s) {
    for (const PencilDev &P : c.host) {
        const int n = P.n;
        const int gy = (n + kGemmT - 1) / kGemmT;
        hipLaunchKernelGGL(k_handoff_gemm, dim3((P.mr + kGemmT - 1) / kGemmT, gy), dim3(256), 0, s,
                           P.mr, n, P.Fw, P.ldf, P.Z32, P.ldz, P.tmp, P.ldf);
        GHSVD_HIP(hipMemcpy2DAsync(P.Fw, P.ldf * sizeof(double2), P.tmp, P.ldf * sizeof(double2),
                                   P.mr * sizeof(double2), n, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_handoff_gemm, dim3((P.pr + kGemmT - 1) / kGemmT, gy), dim3(256), 0, s,
                           P.pr, n, P.Gw, P.ldg, P.Z32, P.ldz, P.tmp, P.ldg);
        GHSVD_HIP(hipMemcpy2DAsync(P.Gw, P.ldg * sizeof(double2), P.tmp, P.ldg * sizeof(double2),
                                   P.pr * sizeof(double2), n, hipMemcpyDeviceToDevice, s));
        int bx = (n + 255) / 256;
        if (bx > 16) bx = 16;
        hipLaunchKernelGGL(k_to_f64, dim3(bx, n), dim3(256), 0, s, n, n, P.Z32, P.ldz, P.Zw, P.ldz);
    }
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

}  // namespace ghsvd
