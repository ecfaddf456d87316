// sweep.hpp -- pointwise sweep machinery shared by the solver entry points.
#pragma once

#include "hz_common.hpp"

namespace ghsvd {

constexpr int kMaxHist = 128;  // sweeps whose counters are kept on the device
// Default sweep cap per stage.  Algorithm 2 uses about 30 for the paper's
// well-conditioned data; the sweep count grows with cond(G^*G) (about 11 at
// 1e2, 29 at 1e16 for n = 256), so the cap leaves room for cond(S) ~ 1e16.
constexpr int kDefaultMaxSweeps = 60;

// Device-side state of one pencil's sweep iteration.  Kernels read `done`
// at entry and return at once when it is set, so work enqueued past
// convergence costs only its launch.
struct SweepState {
    int done;        // 1: converged, capped, or failed
    int sweeps;      // sweeps completed in the current stage
    int err;         // first error status (0 = none)
    int converged;   // 1: the last sweep had no big transformation
    int max_sweeps;  // cap of the current stage
    int noise_floor;  // 1: also stop once a sweep's big count is at most visited / 1024
    int pad[2];
    unsigned long long hist[3 * kMaxHist];  // (visited, transformed, big) per sweep
};

// Arguments of the pair kernels (one pencil, one precision).
struct SweepArgs {
    void *F;     // m x n, complex (double2 or float2), column-major
    long ldf;
    int m;       // rows of F
    int nplus;   // rows 0..nplus-1 carry J = +1, the rest J = -1
    void *G;     // p x n
    long ldg;
    int p;
    void *Z;     // n x n accumulated transformation
    long ldz;
    int n;       // columns
    int N;       // n rounded up to even (round-robin players)
    int nslots;  // N / 2
    double tol;  // eps * sqrt(n)
    int crit;    // criterion form
    int fp32;    // 1: FP32 storage stage
    unsigned long long *slot_cnt;  // [nslots * 3] per-slot counters of the sweep
    SweepState *st;
};

// Launch geometry of the pair kernel.
struct PairGeom {
    int nt;  // threads per pivot pair (64 * waves)
    int r;   // rows held per thread in registers (0: stream the columns twice)
};

using PairFn = void (*)(SweepArgs, int);

// Launches one round-robin step of the pair kernel (with optional event timing).
void launch_pair_step(PairFn fn, const SweepArgs &a, PairGeom g, int step, hipStream_t stream);

struct SweepResult {
    int status;
    int sweeps;
    int converged;
    long long visited, transformed, big;
};


PairGeom choose_pair_geom(int rows, int waves_per_pair);

// Runs up to max_sweeps pointwise sweeps (device-side convergence flag,
// host check after each sweep).  `state` and `slot_cnt` are device buffers
// (one SweepState, nslots * 3 counters).  Synchronizes `stream`.
int run_pointwise_sweeps(SweepArgs a, int max_sweeps, PairGeom g, hipStream_t stream,
                         SweepResult &res);

// Enqueues one pointwise sweep (n - 1 or n steps plus the end-of-sweep
// bookkeeping) without synchronizing.
int enqueue_pointwise_sweep(const SweepArgs &a, PairGeom g, hipStream_t stream);

// End-of-sweep bookkeeping over `nslots` per-slot counters (kernel).
int enqueue_end_sweep(SweepState *st, unsigned long long *cnt, int nslots, hipStream_t stream);

// When the environment variable GHSVD_TRACE is set, prints the per-sweep
// counters of a finished stage to stderr (one line per sweep).
void trace_stage(const char *name, const SweepState &hs);

// Zeroes the state and the per-slot counters (kernel, graph-safe).
// noise_floor = 1 for the FP32 warm-up: stop once the big transformations
// of a sweep are at most 1/1024 of the visited pairs (the pairs still
// rotating then are those FP32 cannot resolve; the FP64 sweeps take over).
int enqueue_reset_state(SweepState *st, unsigned long long *slot_cnt, int nslots,
                        int max_sweeps, hipStream_t stream, int noise_floor = 0);

}  // namespace ghsvd
