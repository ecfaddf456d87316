// sweep.hpp -- sweep stages over a batch of pencils.
#pragma once

#include <vector>

#include "batch.hpp"

namespace ghsvd {

struct SweepResult {
    int status;
    int sweeps;
    int converged;
    long long visited, transformed, big;
};

// Launch geometry of the pointwise pair kernel.
struct PairGeom {
    int nt;  // threads per pivot pair (64 * waves)
    int r;   // rows held per thread in registers (0: stream the columns twice)
};

PairGeom choose_pair_geom(int rows, int waves_per_pair);

// Host view of a batch: the device descriptor array and the prefix sums of
// the workgroups per pencil for each kind of launch.
struct BatchCtx {
    int B = 0;
    PencilDev *dev = nullptr;       // device [B]
    std::vector<PencilDev> host;    // host copy
    int *pre_dev = nullptr;         // device prefix arrays, kKinds blocks of B + 1 ints
    std::vector<int> pre;           // host copy
    enum { kSlots = 0, kCols = 1, kGram = 2, kBp = 3, kUpd = 4, kOne = 5, kKinds = 6 };
    const int *pre_of(int kind) const { return pre_dev + kind * (B + 1); }
    int total(int kind) const { return pre[kind * (B + 1) + B]; }
    int max_n = 0, max_rows = 0;
    int *done_dev = nullptr;        // device [B] stage flags gathered per round
};

// Builds the prefix sums and copies descriptors and sums to the device
// (dev and pre_dev must point at device buffers of the right size).
int upload_batch(BatchCtx &c, hipStream_t s);

// Pointwise sweeps (Algorithm 2 on the round-robin ordering) for every
// pencil of the batch until each converges or hits max_sweeps.  fp32: the
// complex64 copies F32/G32/Z32 (warm-up stage, noise-floor stop).
int run_pointwise_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, PairGeom g,
                        hipStream_t s, std::vector<SweepResult> &res);

// Level-2 blocked sweeps (Section 6.4) for every pencil with n >= 4.
int run_blocked_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, hipStream_t s,
                      std::vector<SweepResult> &res);

// When the environment variable GHSVD_TRACE is set, prints the per-sweep
// counters of a finished stage to stderr (one line per sweep).
void trace_stage(const char *name, int pencil, const SweepState &hs);

// Pair-kernel timing record (see ghsvd_profile_enable).
void prof_before(hipStream_t s, hipEvent_t &e0, hipEvent_t &e1);
void prof_after(hipStream_t s, hipEvent_t e0, hipEvent_t e1);

// Shared host loop of the stages: resets the per-pencil states (blocked = 1
// retires pencils too small for blocking at once), then repeats `one_step`
// (which enqueues one global step for all pencils) in rounds of
// `steps_per_round` until every pencil is done, and collects the results.
using StepFn = int (*)(const BatchCtx &, const void *, hipStream_t);
int drive_stage(const BatchCtx &c, int max_sweeps, int noise_floor, int blocked, StepFn one_step,
                const void *arg, int steps_per_round, const char *name, hipStream_t s,
                std::vector<SweepResult> &res);

// Last-workgroup protocol of a step: every workgroup of a pencil calls this
// at its end (all threads); it returns true in exactly one workgroup, the
// last to finish, which then sees the writes of all the others (the release
// fence before, and the acquire fence after, the counting atomic).
__device__ inline bool last_workgroup(SweepState *st, unsigned total) {
    __shared__ int last_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&st->fin, 1u);
        last_s = (prev + 1u == total) ? 1 : 0;
        if (last_s) __threadfence();
    }
    __syncthreads();
    return last_s != 0;
}

// Run by all threads of the last workgroup of a pencil's step: advances the
// step counter; at the end of a sweep sums the per-slot counters in a fixed
// order, clears them, records them, and sets the stop flags (Section 6.1.7:
// no big transformation in the sweep; Algorithm 2: the sweep cap; the FP32
// noise floor).
__device__ inline void step_done(SweepState *st, unsigned long long *cnt, int nslots, int steps) {
    __shared__ int ls_s;
    __shared__ double red[3 * 16];
    if (threadIdx.x == 0) ls_s = st->lstep + 1;
    __syncthreads();
    const int ls = ls_s;
    if (ls < steps) {
        if (threadIdx.x == 0) {
            st->lstep = ls;
            st->fin = 0u;
        }
        return;
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) {
        v[0] += (double)cnt[3 * k + 0];
        v[1] += (double)cnt[3 * k + 1];
        v[2] += (double)cnt[3 * k + 2];
        cnt[3 * k + 0] = 0ull;
        cnt[3 * k + 1] = 0ull;
        cnt[3 * k + 2] = 0ull;
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        const int sw = st->sweeps;
        if (sw < kMaxHist) {
            st->hist[3 * sw + 0] = (unsigned long long)v[0];
            st->hist[3 * sw + 1] = (unsigned long long)v[1];
            st->hist[3 * sw + 2] = (unsigned long long)v[2];
        }
        st->sweeps = sw + 1;
        if (st->err != 0) {
            st->done = 1;
        } else if (v[2] == 0.0) {
            st->done = 1;
            st->converged = 1;
        } else if (st->noise_floor && v[2] * 1024.0 <= v[0]) {
            st->done = 1;
        } else if (sw + 1 >= st->max_sweeps) {
            st->done = 1;
        }
        st->lstep = 0;
        st->fin = 0u;
    }
}

}  // namespace ghsvd
