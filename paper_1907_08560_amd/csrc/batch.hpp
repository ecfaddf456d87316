// batch.hpp -- device-side description of the pencils a launch works on.
//
// Every sweep and reduction kernel runs over a batch of pencils (one pencil
// for ghsvd_solve): the host writes one PencilDev per pencil into device
// memory, plus prefix sums of the workgroups each pencil needs in a given
// launch; a workgroup finds its pencil by binary search over the prefix sums.
// Per-pencil iteration state lives in device memory (SweepState, JqrState),
// so a round of launches takes the same arguments every time (and can be
// captured into a graph and replayed).
#pragma once

#include "hz_common.hpp"

namespace ghsvd {

constexpr int kMaxHist = 128;  // sweeps whose counters are kept on the device
// Default sweep cap per stage.  Algorithm 2 uses about 30 for the paper's
// well-conditioned data; the sweep count grows with cond(G^*G) (about 11 at
// 1e2, 29 at 1e16 for n = 256), so the cap leaves room for cond(S) ~ 1e16.
constexpr int kDefaultMaxSweeps = 60;

// Iteration state of one pencil in one sweep stage.
struct SweepState {
    int done;        // 1: converged, capped, or failed
    int sweeps;      // sweeps completed in the stage
    int err;         // first error status (0 = none)
    int converged;   // 1: the last sweep had no big transformation
    int max_sweeps;  // cap of the stage
    int noise_floor; // 1: also stop at the noise floor (FP32 stage, see k_end_round)
    int stop_all;    // 1: stop after a sweep with no transformation at all, big or small
                     // (the inner level of a blocked sweep, Section 6.1.7); else no big one
    unsigned long long hist[3 * kMaxHist];  // (visited, transformed, big) per sweep
};

// State of the hyperbolic QR of one pencil (the k-loop runs on the device).
// Two copies, by the parity of the step: a step reads one and its last
// kernel writes the other, so no kernel reads state it may be overwriting.
struct JqrState {
    int k;       // first unreduced column (and row)
    int status;  // 0 or an error
    int n2x2;    // 2x2 pivots taken
    int pad;
};

// Decision of the first Bunch-Kaufman test at the current step (written by
// the second kernel of the step, read by the third).
struct JqrDecision {
    int bi;     // diagonal pivot (logical column) swapped to position k
    int ii;     // candidate column of the second test
    int need2;  // the second test is required
    int pad;
    double lam;  // |h_{k,ii}|
};

struct PencilDev {
    // sizes
    int m, n, p;      // input sizes
    int mr, pr;       // rows of F and G as swept
    int reduce;       // one-time reduction active
    int N, nslots;    // pointwise round robin: players (n rounded up to even), slots
    int w, nb, nbp;   // blocked: block width, block columns (even), block pairs per step
    int kf, kg;       // blocked: Gram chunks over F rows, over G rows
    int tf, tg, tz;   // blocked: 16-row update strips over F, G, Z
    int tu;           // blocked: update workgroups per block pair
    int skip_rank;    // pointwise FP64: a pivot pair whose G columns look dependent is skipped
                      // (left to later sweeps) instead of failing the pencil
    // caller buffers
    const double2 *Fin;
    long ldfin;
    const int8_t *Jin;
    const double2 *Gin;
    long ldgin;
    double *lambda;
    double2 *X;
    long ldx;
    // reduction scratch
    double2 *Ft;
    long ldft;
    double2 *Gt;
    long ldgt;
    JqrState *jst;    // [2] by step parity
    JqrDecision *jdec;
    double *hd;      // J-norm^2 of each physical column over the unreduced rows
    double *hl;      // the same by logical column (position in the step's column order)
    double2 *hc;
    double *hi;
    int *cpb;        // column map after the diagonal-pivot swap of the current step
    double2 *rblk;   // rows k, k+1 of each pivot column at the end of its step (2 n)
    int *pblk;       // first row and size of each column's pivot block (2 n)
    double2 *qdiag;  // R_kk of the QR of G P2 (n)
    double *qnrm;    // ||x|| of the column each QR reflector of G is built from (n)
    int8_t *Jw;       // [2 m] by step parity during the reduction; J_sq in the first copy after
    int *rowmap;
    int *perm;        // column map P2 (logical column j is physical column perm[j] of Ft)
    // sweep buffers
    double2 *Fw;
    long ldf;
    double2 *Gw;
    long ldg;
    double2 *Zw;
    long ldz;
    float2 *F32, *G32, *Z32;
    SweepState *st;
    unsigned long long *slot_cnt;  // pointwise: 3 per slot
    // outputs scratch
    double *lam_tmp, *scale;
    int *rank;
    int *small;  // [0] input flags, [1] n_plus, [2] output flags
    double *gnorm2;
    // blocked scratch
    double2 *part;   // [nbp][kf + kg][PB * PB] partial Grams
    double2 *zh64;   // [nbp][PB * PB]
    float2 *zh32;
    double2 *gp;     // w = 32: [nbp][2][64 * 65 / 2] block-pivot Grams H^, S^, packed upper
    int *ntr;        // [nbp]
    unsigned long long *bcnt;  // [nbp * 3]
    double2 *tmp;    // hand-off product
};

// Pencil of workgroup `blk` given prefix sums pre[0..B] (pre[0] = 0).
// Index of workgroup blk within its pencil's range of a launch (pencil 0
// starts at 0, which saves a memory access in the common one-pencil case).
__device__ __forceinline__ int pencil_local(const int *pre, int pk, int blk) {
    return pk ? blk - pre[pk] : blk;
}

// The pencil is the last p with pre[p] <= blk (a pencil with no workgroups
// in the launch has pre[p] == pre[p + 1]).  Up to kFindWide pencils, every
// wavefront counts those p with one load per lane and chunk of 64 and a
// ballot (one memory latency instead of a chain of dependent ones); larger
// batches take the binary search.  Must be called by whole wavefronts.
constexpr int kFindWide = 1024;

__device__ __forceinline__ int find_pencil(const int *pre, int B, int blk) {
    if (B <= 1) return 0;
    if (B <= kFindWide) {
        const int lane = threadIdx.x & (kWave - 1);
        int cnt = 0;
        for (int c = 0; c < B; c += kWave) {
            const int p = c + lane;
            cnt += __popcll(__ballot(p < B && pre[p] <= blk));
        }
        return cnt - 1;
    }
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace ghsvd
