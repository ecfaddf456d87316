// sweep.hpp -- sweep stages over a batch of pencils.
#pragma once

#include <hip/hip_ext.h>

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
    int *win_dev = nullptr;         // device: reduction column windows, 2 kWinRows blocks of B + 1
    std::vector<int> win;           // host copy (built by the reduction)
    int *done_dev = nullptr;        // device [2 (B + 1)] small per-pencil results for the host
    int *flag_dev = nullptr;        // device [B] 1: the pencil's sweep stage is done (read by
                                    // every sweep kernel, written at the end of each round)
    bool plain = false;             // launch rounds directly on the caller's stream: no
                                    // captured graph, internal stream or timing events
    int stop_all = 0;               // the stage stops a pencil after a sweep with no
                                    // transformation at all (else: no big one)
    char *short_buf = nullptr;      // workspace region of the (J)QR-shortened blocked stage
    size_t short_cap = 0;
};

// Rows of the reduction's column-window table (see run_reduction).
constexpr int kWinRows = 64;

// Builds the prefix sums and copies descriptors and sums to the device
// (dev and pre_dev must point at device buffers of the right size).
int upload_batch(BatchCtx &c, hipStream_t s);

// Pointwise sweeps (Algorithm 2 on the round-robin ordering) for every
// pencil of the batch until each converges or hits max_sweeps.  fp32: the
// complex64 copies F32/G32/Z32 (warm-up stage, noise-floor stop).
// presolved (host, may be NULL): pencils marked 1 start the stage converged.
int run_pointwise_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, PairGeom g,
                        hipStream_t s, std::vector<SweepResult> &res,
                        const std::vector<int> *presolved = nullptr);

// Level-2 blocked sweeps (Section 6.4) for every pencil with n >= 4.
// presolved as for run_pointwise_stage.
int run_blocked_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, int inner_order,
                      hipStream_t s, std::vector<SweepResult> &res,
                      const std::vector<int> *presolved = nullptr);

// When the environment variable GHSVD_TRACE is set, prints the per-sweep
// counters of a finished stage to stderr (one line per sweep).
void trace_stage(const char *name, int pencil, const SweepState &hs);

// Sweep-kernel timing record (see ghsvd_profile_enable), per kernel kind.
enum { kProfPair64 = 0, kProfPair32 = 1, kProfGram = 2, kProfInner = 3, kProfUpdate = 4,
       kProfGram32 = 5, kProfInner32 = 6, kProfUpdate32 = 7, kProfReduce = 8, kProfKinds = 9 };
// prof_take decides whether this launch of `kind` is sampled and, if so,
// hands out two events (else nullptr) for the launch itself to record at the
// kernel's start and end (launch_ev); prof_done files the pair.
void prof_take(int kind, hipEvent_t &e0, hipEvent_t &e1);
void prof_done(int kind, hipEvent_t e0, hipEvent_t e1);

// A kernel launch that records e0 as the kernel starts and e1 as it ends
// (hipExtLaunchKernelGGL), so a sampled duration is the kernel's own; with
// no events it is a plain launch (also under graph capture).
template <typename F, typename... Args>
inline void launch_ev(F k, dim3 g, dim3 b, uint32_t shm, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1, Args... args) {
    if (e0 || e1) hipExtLaunchKernelGGL(k, g, b, shm, s, e0, e1, 0, args...);
    else hipLaunchKernelGGL(k, g, b, shm, s, args...);
}

// Shared host loop of the stages: resets the per-pencil states (blocked = 1
// retires pencils too small for blocking at once), then runs rounds until
// every pencil is done.  A round is one sweep of every pencil still running:
// `one_step(c, arg, i, s)` for i = 0 .. steps_per_round - 1 (it enqueues
// global step i for all pencils; a pencil with fewer steps per sweep idles
// in the surplus steps), then the end-of-round kernel, which applies the
// stopping rules.  The round is captured once into a graph on an internal
// stream and replayed (unless kernel timing is on or GHSVD_NO_GRAPH is set).
using StepFn = int (*)(const BatchCtx &, const void *, int, hipStream_t);
int drive_stage(const BatchCtx &c, int max_sweeps, int noise_floor, int blocked, StepFn one_step,
                const void *arg, int steps_per_round, const char *name, hipStream_t s,
                std::vector<SweepResult> &res, const std::vector<int> *presolved = nullptr);

}  // namespace ghsvd
