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

#include "hz_step.hpp"
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
constexpr int kGramSub = 64;     // rows staged in LDS at a time
constexpr int kUpdRows = 64;     // rows of one update tile

struct BlkArgs {
    void *F;
    long ldf;
    int m;
    int nplus;
    void *G;
    long ldg;
    int p;
    void *Z;
    long ldz;
    int n;
    int w;    // block width
    int nb;   // block columns (even)
    int nbp;  // block pairs per step
    int kf, kg;          // Gram chunks over F rows, over G rows
    int tf, tg, tz;      // update tiles over F, G, Z rows
    double eps;          // machine precision of (6.12) for the inner level
    int crit;
    int fp32;
    double2 *part;       // [nbp][kf + kg][PB * PB] partial Grams
    double2 *zh64;       // [nbp][PB * PB] accumulated inner transforms
    float2 *zh32;        // same in FP32 (FP32 stage)
    int *ntr;            // [nbp] inner transformations of the current step
    unsigned long long *cnt;  // [nbp * 3] per-slot counters of the block sweep
    SweepState *st;
};

__device__ __forceinline__ int blk_width(int n, int w, int b) {
    const int c = n - b * w;
    return c < 0 ? 0 : (c > w ? w : c);
}

// Global column of pivot column cc (block a's columns, then block b's).
__device__ __forceinline__ int blk_col(int w, int a, int b, int ca, int cc) {
    return cc < ca ? a * w + cc : b * w + (cc - ca);
}

template <typename T, int PB>
__global__ __launch_bounds__(256) void k_blk_gram(BlkArgs A, int step) {
    using C2 = typename Mfma<T>::c2;
    using ACC = typename Mfma<T>::acc;
    constexpr int NTD = PB / 16;          // output tiles per dimension
    constexpr int NT2 = NTD * NTD;        // output tiles
    constexpr int KSPLIT = 4 / NT2;       // waves sharing one output tile
    __shared__ C2 tile[kGramSub][PB + 1];
    __shared__ double2 red[KSPLIT > 1 ? 4 * 256 : 1];
    if (A.st->done) return;
    const int bpi = blockIdx.x, kc = blockIdx.y;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) return;
    const bool isF = kc < A.kf;
    const int r0 = (isF ? kc : kc - A.kf) * kGramChunk;
    const int rows = isF ? A.m : A.p;
    const long ld = isF ? A.ldf : A.ldg;
    const C2 *X = reinterpret_cast<const C2 *>(isF ? A.F : A.G);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int t = wv % NT2, ks = wv / NT2;
    const int ti = t % NTD, tj = t / NTD;
    ACC acc_re = {0, 0, 0, 0}, acc_im = {0, 0, 0, 0};
    for (int s0 = r0; s0 < r0 + kGramChunk && s0 < rows; s0 += kGramSub) {
        for (int idx = tid; idx < kGramSub * PB; idx += 256) {
            const int cc = idx / kGramSub, rr = idx % kGramSub;
            C2 v;
            v.x = 0;
            v.y = 0;
            if (cc < c && s0 + rr < rows) v = X[(size_t)blk_col(A.w, a, b, ca, cc) * ld + s0 + rr];
            tile[rr][cc] = v;
        }
        __syncthreads();
        constexpr int KW = kGramSub / KSPLIT;
        for (int k0 = ks * KW; k0 < ks * KW + KW; k0 += 4) {
            const int k = k0 + (lane >> 4);
            const C2 fa = tile[k][ti * 16 + (lane & 15)];
            C2 fb = tile[k][tj * 16 + (lane & 15)];
            if (isF && s0 + k >= A.nplus) {
                fb.x = -fb.x;
                fb.y = -fb.y;
            }
            // conj(fa) * fb
            acc_re = Mfma<T>::mma(fa.x, fb.x, acc_re);
            acc_re = Mfma<T>::mma(fa.y, fb.y, acc_re);
            acc_im = Mfma<T>::mma(fa.x, fb.y, acc_im);
            acc_im = Mfma<T>::mma(-fa.y, fb.x, acc_im);
        }
        __syncthreads();
    }
    double2 *P = A.part + ((size_t)bpi * (A.kf + A.kg) + kc) * PB * PB;
    if constexpr (KSPLIT > 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wv * 256 + r * 64 + lane] = cmk((double)acc_re[r], (double)acc_im[r]);
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double2 s = red[r * 64 + lane];
                for (int q = 1; q < KSPLIT; ++q) s = cadd(s, red[q * 256 + r * 64 + lane]);
                const int i = ti * 16 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
                P[(size_t)j * PB + i] = s;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = ti * 16 + Mfma<T>::row(lane, r), j = tj * 16 + (lane & 15);
            P[(size_t)j * PB + i] = cmk((double)acc_re[r], (double)acc_im[r]);
        }
    }
}

// One inner sweep over the block pivot (H^, S^) in LDS.  An inner step:
// (a) one lane per pivot pair computes the FP64 2x2 step; (b) every thread
// takes one 2x2 block (rows of pair k, columns of pair k') and applies
// H <- Z_k^* H Z_k', S <- Z_k^* S Z_k', Zs <- Zs Z_k' to it.  The pairs of a
// step are disjoint, so the blocks are independent and the two-sided update
// needs a single pass over H and S.  Pair slots whose second column is a bye
// or padding (>= c) carry the identity; padding entries are zero and stay so.
template <int PB>
__global__ __launch_bounds__(256) void k_blk_inner(BlkArgs A, int step) {
    constexpr int NP = PB / 2;   // pivot pair slots per inner step
    constexpr int NB = NP * NP;  // 2x2 blocks
    __shared__ double2 H[PB][PB + 1];
    __shared__ double2 S[PB][PB + 1];
    __shared__ double2 Zs[PB][PB + 1];
    __shared__ double2 zpar[NP][4];
    __shared__ int pq_s[NP][2];
    __shared__ int act_s[NP];
    __shared__ double red[3 * 4];
    if (A.st->done) return;
    const int bpi = blockIdx.x;
    const int tid = threadIdx.x;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) {
        if (tid == 0) A.ntr[bpi] = 0;
        return;
    }
    const int KC = A.kf + A.kg;
    const double2 *P = A.part + (size_t)bpi * KC * PB * PB;
    for (int idx = tid; idx < PB * PB; idx += 256) {
        const int i = idx % PB, j = idx / PB;
        double2 h = cmk(0.0, 0.0), s = cmk(0.0, 0.0);
        for (int k = 0; k < A.kf; ++k) h = cadd(h, P[(size_t)k * PB * PB + idx]);
        for (int k = A.kf; k < KC; ++k) s = cadd(s, P[(size_t)k * PB * PB + idx]);
        H[i][j] = h;
        S[i][j] = s;
        Zs[i][j] = cmk(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int C = c + (c & 1);
    const int islots = C / 2;
    const double tol = A.eps * sqrt((double)c);
    double cv = 0.0, ct = 0.0, cbig = 0.0;
    for (int s = 0; s < C - 1; ++s) {
        if (tid < NP) {
            int pp = -1, qq = -1, kind = kSkip;
            if (tid < islots) {
                rr_pair(C, s, tid, pp, qq);
                if (qq < c) {
                    Zp z;
                    kind = hz_step_fast(H[pp][pp].x, H[qq][qq].x, H[pp][qq], S[pp][pp].x,
                                        S[qq][qq].x, S[pp][qq], tol, A.crit, z, A.fp32);
                    cv += 1.0;
                    if (kind == GHSVD_ENONFINITE) atomicCAS(&A.st->err, 0, GHSVD_ENONFINITE);
                    if (kind < 0) kind = kSkip;  // dependent-looking pivot: left to the finish
                    zpar[tid][0] = z.z11;
                    zpar[tid][1] = z.z21;
                    zpar[tid][2] = z.z12;
                    zpar[tid][3] = z.z22;
                    ct += kind > 0 ? 1.0 : 0.0;
                    cbig += kind == kBig ? 1.0 : 0.0;
                }
            }
            pq_s[tid][0] = pp;
            pq_s[tid][1] = qq;
            act_s[tid] = kind > 0;
        }
        __syncthreads();
        for (int blk = tid; blk < NB; blk += 256) {
            const int kr = blk % NP, kc = blk / NP;  // row pair, column pair
            const int p1 = pq_s[kr][0], q1 = pq_s[kr][1];
            const int p2 = pq_s[kc][0], q2 = pq_s[kc][1];
            const bool ar = act_s[kr], ac = act_s[kc];
            if (p1 < 0 || p2 < 0 || (!ar && !ac)) continue;  // padding slot or identity
            // loads first (one LDS round trip), then arithmetic, then stores
            const double2 one = cmk(1.0, 0.0), zero = cmk(0.0, 0.0);
            double2 zr[4], zc[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                zr[e] = zpar[kr][e];
                zc[e] = zpar[kc][e];
            }
            const double2 h11 = H[p1][p2], h12 = H[p1][q2], h21 = H[q1][p2], h22 = H[q1][q2];
            const double2 s11 = S[p1][p2], s12 = S[p1][q2], s21 = S[q1][p2], s22 = S[q1][q2];
            const double2 w11 = Zs[p1][p2], w12 = Zs[p1][q2], w21 = Zs[q1][p2], w22 = Zs[q1][q2];
            const double2 r11 = ar ? zr[0] : one, r21 = ar ? zr[1] : zero;
            const double2 r12 = ar ? zr[2] : zero, r22 = ar ? zr[3] : one;
            const double2 c11 = ac ? zc[0] : one, c21 = ac ? zc[1] : zero;
            const double2 c12 = ac ? zc[2] : zero, c22 = ac ? zc[3] : one;
            // M_blk <- R^* M_blk Cz for H and S; Zs_blk <- Zs_blk Cz
            double2 x11 = cadd(cmul(h11, c11), cmul(h12, c21));
            double2 x12 = cadd(cmul(h11, c12), cmul(h12, c22));
            double2 x21 = cadd(cmul(h21, c11), cmul(h22, c21));
            double2 x22 = cadd(cmul(h21, c12), cmul(h22, c22));
            const double2 H11 = cadd(cmulc(r11, x11), cmulc(r21, x21));
            const double2 H12 = cadd(cmulc(r11, x12), cmulc(r21, x22));
            const double2 H21 = cadd(cmulc(r12, x11), cmulc(r22, x21));
            const double2 H22 = cadd(cmulc(r12, x12), cmulc(r22, x22));
            x11 = cadd(cmul(s11, c11), cmul(s12, c21));
            x12 = cadd(cmul(s11, c12), cmul(s12, c22));
            x21 = cadd(cmul(s21, c11), cmul(s22, c21));
            x22 = cadd(cmul(s21, c12), cmul(s22, c22));
            const double2 S11 = cadd(cmulc(r11, x11), cmulc(r21, x21));
            const double2 S12 = cadd(cmulc(r11, x12), cmulc(r21, x22));
            const double2 S21 = cadd(cmulc(r12, x11), cmulc(r22, x21));
            const double2 S22 = cadd(cmulc(r12, x12), cmulc(r22, x22));
            const double2 W11 = cadd(cmul(w11, c11), cmul(w12, c21));
            const double2 W12 = cadd(cmul(w11, c12), cmul(w12, c22));
            const double2 W21 = cadd(cmul(w21, c11), cmul(w22, c21));
            const double2 W22 = cadd(cmul(w21, c12), cmul(w22, c22));
            H[p1][p2] = H11;
            H[p1][q2] = H12;
            H[q1][p2] = H21;
            H[q1][q2] = H22;
            S[p1][p2] = S11;
            S[p1][q2] = S12;
            S[q1][p2] = S21;
            S[q1][q2] = S22;
            Zs[p1][p2] = W11;
            Zs[p1][q2] = W12;
            Zs[q1][p2] = W21;
            Zs[q1][q2] = W22;
        }
        __syncthreads();
    }
    double v[3] = {cv, ct, cbig};
    block_sum<3>(v, red);
    double2 *Z64 = A.zh64 + (size_t)bpi * PB * PB;
    float2 *Z32 = A.zh32 ? A.zh32 + (size_t)bpi * PB * PB : nullptr;
    for (int idx = tid; idx < PB * PB; idx += 256) {
        const int i = idx % PB, j = idx / PB;
        const double2 z = Zs[i][j];
        Z64[idx] = z;
        if (Z32) Z32[idx] = make_float2((float)z.x, (float)z.y);
    }
    if (tid == 0) {
        A.ntr[bpi] = (int)v[1];
        unsigned long long *cn = A.cnt + 3 * bpi;
        cn[0] += (unsigned long long)v[0];
        cn[1] += (unsigned long long)v[1];
        cn[2] += (unsigned long long)v[2];
    }
}

template <typename T, int PB>
__global__ __launch_bounds__(256) void k_blk_update(BlkArgs A, int step) {
    using C2 = typename Mfma<T>::c2;
    using ACC = typename Mfma<T>::acc;
    constexpr int NTJ = PB / 16;
    constexpr int NTI = kUpdRows / 16;
    constexpr int TILES = NTI * NTJ;
    __shared__ C2 Xs[kUpdRows][PB + 1];
    __shared__ C2 Zh[PB][PB + 1];
    if (A.st->done) return;
    const int bpi = blockIdx.x;
    if (A.ntr[bpi] == 0) return;
    int a, b;
    rr_pair(A.nb, step, bpi, a, b);
    const int ca = blk_width(A.n, A.w, a), cb = blk_width(A.n, A.w, b);
    const int c = ca + cb;
    if (c < 2) return;
    int t = blockIdx.y;
    C2 *X;
    long ld;
    int rows;
    if (t < A.tf) {
        X = reinterpret_cast<C2 *>(A.F);
        ld = A.ldf;
        rows = A.m;
    } else if (t < A.tf + A.tg) {
        t -= A.tf;
        X = reinterpret_cast<C2 *>(A.G);
        ld = A.ldg;
        rows = A.p;
    } else {
        t -= A.tf + A.tg;
        X = reinterpret_cast<C2 *>(A.Z);
        ld = A.ldz;
        rows = A.n;
    }
    const int r0 = t * kUpdRows;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int idx = tid; idx < PB * PB; idx += 256) {
        const int k = idx % PB, j = idx / PB;
        C2 z;
        if constexpr (sizeof(T) == 8) {
            z = A.zh64[(size_t)bpi * PB * PB + idx];
        } else {
            z = A.zh32[(size_t)bpi * PB * PB + idx];
        }
        Zh[k][j] = z;
    }
    for (int idx = tid; idx < kUpdRows * PB; idx += 256) {
        const int cc = idx / kUpdRows, rr = idx % kUpdRows;
        C2 v;
        v.x = 0;
        v.y = 0;
        if (cc < c && r0 + rr < rows) v = X[(size_t)blk_col(A.w, a, b, ca, cc) * ld + r0 + rr];
        Xs[rr][cc] = v;
    }
    __syncthreads();
    ACC out_re[(TILES + 3) / 4], out_im[(TILES + 3) / 4];
#pragma unroll
    for (int q = 0; q < (TILES + 3) / 4; ++q) {
        const int tt = wv + 4 * q;
        out_re[q] = ACC{0, 0, 0, 0};
        out_im[q] = ACC{0, 0, 0, 0};
        if (tt >= TILES) continue;
        const int ti = tt % NTI, tj = tt / NTI;
        for (int k0 = 0; k0 < PB; k0 += 4) {
            const int k = k0 + (lane >> 4);
            const C2 xa = Xs[ti * 16 + (lane & 15)][k];
            const C2 zb = Zh[k][tj * 16 + (lane & 15)];
            out_re[q] = Mfma<T>::mma(xa.x, zb.x, out_re[q]);
            out_re[q] = Mfma<T>::mma(-xa.y, zb.y, out_re[q]);
            out_im[q] = Mfma<T>::mma(xa.x, zb.y, out_im[q]);
            out_im[q] = Mfma<T>::mma(xa.y, zb.x, out_im[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (TILES + 3) / 4; ++q) {
        const int tt = wv + 4 * q;
        if (tt >= TILES) continue;
        const int ti = tt % NTI, tj = tt / NTI;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            C2 v;
            v.x = out_re[q][r];
            v.y = out_im[q][r];
            Xs[ti * 16 + Mfma<T>::row(lane, r)][tj * 16 + (lane & 15)] = v;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < kUpdRows * PB; idx += 256) {
        const int cc = idx / kUpdRows, rr = idx % kUpdRows;
        if (cc < c && r0 + rr < rows) X[(size_t)blk_col(A.w, a, b, ca, cc) * ld + r0 + rr] = Xs[rr][cc];
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
struct BlkGeom {
    int w, PB, nb, nbp, kf, kg, tf, tg, tz;
};

static BlkGeom blk_geom(int m, int n, int p, int w) {
    BlkGeom g{};
    g.w = w;
    g.PB = 2 * w;
    g.nb = (n + w - 1) / w;
    if (g.nb & 1) g.nb += 1;
    g.nbp = g.nb / 2;
    g.kf = (m + kGramChunk - 1) / kGramChunk;
    g.kg = (p + kGramChunk - 1) / kGramChunk;
    g.tf = (m + kUpdRows - 1) / kUpdRows;
    g.tg = (p + kUpdRows - 1) / kUpdRows;
    g.tz = (n + kUpdRows - 1) / kUpdRows;
    return g;
}

int pick_block_width(int n, int requested) {
    if (requested == 8 || requested == 16) return requested;
    return n >= 512 ? 16 : 8;
}

struct BlkWs {
    double2 *part;
    double2 *zh64;
    float2 *zh32;
    int *ntr;
    unsigned long long *cnt;
    double2 *tmp;  // hand-off product (rows x n)
};

static BlkWs carve_blk(Carver &c, const Plan &pl, int w) {
    BlkWs b{};
    const BlkGeom g = blk_geom(pl.mr, pl.n, pl.pr, w);
    const size_t pb2 = (size_t)g.PB * g.PB;
    b.part = c.take<double2>((size_t)g.nbp * (g.kf + g.kg) * pb2);
    b.zh64 = c.take<double2>((size_t)g.nbp * pb2);
    b.zh32 = c.take<float2>((size_t)g.nbp * pb2);
    b.ntr = c.take<int>(g.nbp);
    b.cnt = c.take<unsigned long long>(3 * (size_t)g.nbp);
    if (pl.mixed) {
        const long ld = pl.ldf > pl.ldg ? pl.ldf : pl.ldg;
        b.tmp = c.take<double2>((size_t)ld * pl.n);
    }
    return b;
}

void carve_blocked(Carver &c, const Plan &pl, PencilWs &w) {
    // sized for the widest block choice
    Carver probe{nullptr, 0, (size_t)-1};
    (void)carve_blk(probe, pl, 16);
    const size_t need = probe.used;
    w.blk = c.take<char>(need);
    w.blk_bytes = need;
}

static BlkWs blk_ws(const Plan &pl, const PencilWs &w, int width) {
    Carver c{reinterpret_cast<char *>(w.blk), 0, w.blk_bytes};
    return carve_blk(c, pl, width);
}

using BlkFn = void (*)(BlkArgs, int);

static int run_blocked_sweeps(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                              int fp32, hipStream_t s, SweepResult &res) {
    res = SweepResult{GHSVD_OK, 0, 0, 0, 0, 0};
    const int width = pick_block_width(pl.n, o.block_width);
    const BlkGeom g = blk_geom(pl.mr, pl.n, pl.pr, width);
    const BlkWs bw = blk_ws(pl, w, width);
    BlkArgs A{};
    A.F = fp32 ? (void *)w.F32 : (void *)w.Fw;
    A.ldf = pl.ldf;
    A.m = pl.mr;
    A.nplus = nplus;
    A.G = fp32 ? (void *)w.G32 : (void *)w.Gw;
    A.ldg = pl.ldg;
    A.p = pl.pr;
    A.Z = fp32 ? (void *)w.Z32 : (void *)w.Zw;
    A.ldz = pl.ldz;
    A.n = pl.n;
    A.w = g.w;
    A.nb = g.nb;
    A.nbp = g.nbp;
    A.kf = g.kf;
    A.kg = g.kg;
    A.tf = g.tf;
    A.tg = g.tg;
    A.tz = g.tz;
    A.eps = fp32 ? 0x1p-23 : 0x1p-52;
    A.crit = o.crit_literal;
    A.fp32 = fp32;
    A.part = bw.part;
    A.zh64 = bw.zh64;
    A.zh32 = fp32 ? bw.zh32 : nullptr;
    A.ntr = bw.ntr;
    A.cnt = bw.cnt;
    A.st = w.st;
    BlkFn gram, inner, upd;
    if (g.PB == 32) {
        gram = fp32 ? k_blk_gram<float, 32> : k_blk_gram<double, 32>;
        inner = k_blk_inner<32>;
        upd = fp32 ? k_blk_update<float, 32> : k_blk_update<double, 32>;
    } else {
        gram = fp32 ? k_blk_gram<float, 16> : k_blk_gram<double, 16>;
        inner = k_blk_inner<16>;
        upd = fp32 ? k_blk_update<float, 16> : k_blk_update<double, 16>;
    }
    int rc = enqueue_reset_state(w.st, bw.cnt, g.nbp, o.max_sweeps, s, fp32);
    if (rc) return rc;
    SweepState hs;
    for (int sw = 0; sw < o.max_sweeps; ++sw) {
        for (int step = 0; step < g.nb - 1; ++step) {
            hipLaunchKernelGGL(gram, dim3(g.nbp, g.kf + g.kg), dim3(256), 0, s, A, step);
            hipLaunchKernelGGL(inner, dim3(g.nbp), dim3(256), 0, s, A, step);
            hipLaunchKernelGGL(upd, dim3(g.nbp, g.tf + g.tg + g.tz), dim3(256), 0, s, A, step);
        }
        GHSVD_HIP(hipGetLastError());
        if ((rc = enqueue_end_sweep(w.st, bw.cnt, g.nbp, s))) return rc;
        GHSVD_HIP(hipMemcpyAsync(&hs, w.st, offsetof(SweepState, hist), hipMemcpyDeviceToHost, s));
        GHSVD_HIP(hipStreamSynchronize(s));
        if (hs.done) break;
    }
    GHSVD_HIP(hipMemcpyAsync(&hs, w.st, sizeof(SweepState), hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    trace_stage(fp32 ? "blocked-fp32" : "blocked-fp64", hs);
    res.sweeps = hs.sweeps;
    res.converged = hs.converged;
    for (int k = 0; k < hs.sweeps && k < kMaxHist; ++k) {
        res.visited += (long long)hs.hist[3 * k + 0];
        res.transformed += (long long)hs.hist[3 * k + 1];
        res.big += (long long)hs.hist[3 * k + 2];
    }
    res.status = hs.err ? hs.err : (hs.converged ? GHSVD_OK : GHSVD_NOT_CONVERGED);
    return res.status < 0 ? res.status : GHSVD_OK;
}

int run_blocked_fp64(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                     ghsvd_info &info, hipStream_t s) {
    if (pl.n < 4) return GHSVD_OK;
    SweepResult r;
    const int rc = run_blocked_sweeps(pl, w, nplus, o, 0, s, r);
    info.sweeps_fp64 += r.sweeps;
    info.sweeps_blocked += r.sweeps;
    info.pairs_visited += r.visited;
    info.pairs_transformed += r.transformed;
    info.pairs_big += r.big;
    return rc;
}

int run_fp32_stage(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                   ghsvd_info &info, hipStream_t s) {
    const int n = pl.n;
    int bx = (pl.mr + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_to_f32, dim3(bx, n), dim3(256), 0, s, pl.mr, n, w.Fw, pl.ldf, w.F32, pl.ldf);
    bx = (pl.pr + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_to_f32, dim3(bx, n), dim3(256), 0, s, pl.pr, n, w.Gw, pl.ldg, w.G32, pl.ldg);
    int rc = set_identity(n, w.Z32, pl.ldz, 1, s);
    if (rc) return rc;
    SweepResult r{};
    if (o.variant == GHSVD_BLOCKED && n >= 4) {
        rc = run_blocked_sweeps(pl, w, nplus, o, 1, s, r);
        info.sweeps_blocked += r.sweeps;
    } else {
        SweepArgs a = sweep_args(pl, w, nplus, o, 1);
        const int rows = pl.mr > pl.pr ? pl.mr : pl.pr;
        rc = run_pointwise_sweeps(a, o.max_sweeps, choose_pair_geom(rows, o.waves_per_pair), s, r);
        if (rc > 0) rc = GHSVD_OK;
    }
    info.sweeps_fp32 += r.sweeps;
    info.pairs_visited += r.visited;
    info.pairs_transformed += r.transformed;
    info.pairs_big += r.big;
    if (rc < 0) return rc;
    // Hand-off: F <- F Z32, G <- G Z32 in FP64, Z <- Z32.
    const BlkWs bw = blk_ws(pl, w, pick_block_width(n, o.block_width));
    const dim3 gz((n + kGemmT - 1) / kGemmT, (n + kGemmT - 1) / kGemmT);
    hipLaunchKernelGGL(k_handoff_gemm, dim3((pl.mr + kGemmT - 1) / kGemmT, gz.y), dim3(256), 0, s,
                       pl.mr, n, w.Fw, pl.ldf, w.Z32, pl.ldz, bw.tmp, pl.ldf);
    GHSVD_HIP(hipMemcpy2DAsync(w.Fw, pl.ldf * sizeof(double2), bw.tmp, pl.ldf * sizeof(double2),
                               pl.mr * sizeof(double2), n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_handoff_gemm, dim3((pl.pr + kGemmT - 1) / kGemmT, gz.y), dim3(256), 0, s,
                       pl.pr, n, w.Gw, pl.ldg, w.Z32, pl.ldz, bw.tmp, pl.ldg);
    GHSVD_HIP(hipMemcpy2DAsync(w.Gw, pl.ldg * sizeof(double2), bw.tmp, pl.ldg * sizeof(double2),
                               pl.pr * sizeof(double2), n, hipMemcpyDeviceToDevice, s));
    bx = (n + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_to_f64, dim3(bx, n), dim3(256), 0, s, n, n, w.Z32, pl.ldz, w.Zw, pl.ldz);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

}  // namespace ghsvd

using namespace ghsvd;

extern "C" int ghsvd_block_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G,
                                  int ldg, double *Z, int ldz, int block_width, int nsweeps,
                                  int crit_literal, long long *counters, int *sweeps_done,
                                  void *stream) {
    if (n < 4 || m < 1 || p < 1 || ldf < m || ldg < p || ldz < n || nsweeps < 1 ||
        nsweeps > kMaxHist || n_plus < 0 || n_plus > m || !F || !G || !Z)
        return GHSVD_EINVAL;
    if (block_width != 0 && block_width != 8 && block_width != 16) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ghsvd_options o;
    ghsvd_default_options(&o);
    o.block_width = block_width;
    o.max_sweeps = nsweeps;
    o.crit_literal = crit_literal;
    o.variant = GHSVD_BLOCKED;
    Plan pl{};
    pl.m = m;
    pl.n = n;
    pl.p = p;
    pl.mr = m;
    pl.pr = p;
    pl.ldf = ldf;
    pl.ldg = ldg;
    pl.ldz = ldz;
    pl.N = n + (n & 1);
    pl.blocked = 1;
    Carver probe{nullptr, 0, (size_t)-1};
    PencilWs w{};
    w.st = probe.take<SweepState>(1);
    carve_blocked(probe, pl, w);
    void *buf = nullptr;
    GHSVD_HIP(hipMalloc(&buf, probe.used));
    Carver c{reinterpret_cast<char *>(buf), 0, probe.used};
    w.st = c.take<SweepState>(1);
    carve_blocked(c, pl, w);
    w.Fw = reinterpret_cast<double2 *>(F);
    w.Gw = reinterpret_cast<double2 *>(G);
    w.Zw = reinterpret_cast<double2 *>(Z);
    SweepResult r;
    int rc = run_blocked_sweeps(pl, w, n_plus, o, 0, s, r);
    SweepState hs;
    if (hipMemcpy(&hs, w.st, sizeof(SweepState), hipMemcpyDeviceToHost) == hipSuccess) {
        if (counters)
            for (int k = 0; k < nsweeps; ++k)
                for (int j = 0; j < 3; ++j)
                    counters[3 * k + j] = k < hs.sweeps ? (long long)hs.hist[3 * k + j] : 0;
        if (sweeps_done) *sweeps_done = hs.sweeps;
    }
    (void)hipFree(buf);
    return rc < 0 ? rc : r.status;
}
