// solver.hpp -- per-pencil plan, workspace carving and the batch pipeline.
#pragma once

#include <vector>

#include "batch.hpp"
#include "sweep.hpp"

namespace ghsvd {

// Host-side plan of one pencil.
struct Plan {
    int m, n, p;       // input sizes
    int reduce;        // run the one-time reduction
    int mr, pr;        // rows of F and G as swept
    long ldft, ldgt;   // tall scratch copies
    long ldf, ldg, ldz;
    int N;             // n rounded up to even
    int mixed;         // FP32 warm-up stage
    int blocked;       // Level-2 blocked stage
    int w;             // block width (blocked or mixed)
    int inplace;       // the sweep buffers F, G, Z are the caller's: carve no copies
};

Plan make_plan(int m, int n, int p, const ghsvd_options &o, int block_width);
// Carves one pencil's workspace and fills the sizes and scratch pointers of d
// (the caller's buffers are set separately).
void carve_pencil(Carver &c, const Plan &pl, PencilDev &d);
size_t pencil_bytes(const Plan &pl);
// Device bytes shared by a batch of B pencils (descriptors, prefix sums, flags).
size_t batch_bytes(int B);
int pick_block_width(int max_n, int requested);
void fill_options(const ghsvd_options *opt, ghsvd_options &o);

// One pencil's inputs and outputs (device pointers).
struct PencilIO {
    int m, n, p;
    const double2 *F;
    long ldf;
    const int8_t *J;
    const double2 *G;
    long ldg;
    double *lambda;
    double2 *X;
    long ldx;
};

// Timing of the FP64 sweep stages, for the tuner: when passed to solve_batch,
// the blocked and pointwise FP64 stages are bracketed by events (ms, 0 when
// the stage did not run) and the outputs are not formed.
struct StageClock {
    float blocked_ms = 0.0f;
    float pointwise_ms = 0.0f;
};

// The whole path for a batch: input checks, reduction, sweep stages, outputs.
// status[k] and info[k] per pencil; returns the worst status.
int solve_batch(const std::vector<PencilIO> &io, const ghsvd_options &o, void *work, size_t lwork,
                std::vector<ghsvd_info> &info, hipStream_t s, StageClock *clk = nullptr);
size_t solve_batch_bytes(const std::vector<PencilIO> &io, const ghsvd_options &o);

// Device bytes shared by a batch of B pencils, carved from c.
void carve_batch(Carver &c, BatchCtx &bc, int B);

// Block-column update kernel (FP64) of block width w (blocked.hip), for the
// shortened stage.
using BlkFn = void (*)(const PencilDev *, const int *, const int *, int, int);
BlkFn block_update_kernel(int w);

// Blocked FP64 stage with (J)QR-shortened block pivots (shorten.hip): fb = 1
// runs the Full Block inner level; ml = 1 sweeps each shortened pivot with
// the Level-2 blocked stage of width kMlWidth instead of pointwise sweeps
// (three levels).  Needs c.short_buf of short_stage_bytes (which covers both).
int run_blocked_shortened(const BatchCtx &c, int max_sweeps, int crit, int fb, int ml,
                          hipStream_t s, std::vector<SweepResult> &res);
size_t short_stage_bytes(const std::vector<Plan> &outer, int w);
constexpr int kShortFbSweeps = 30;  // C_max of the FB inner level
constexpr int kMlWidth = 8;         // block width of the nested Level-2 stage
inline bool inner_multilevel(int inner_order) {
    return inner_order == GHSVD_INNER_ML_BO || inner_order == GHSVD_INNER_ML_FB;
}
inline bool inner_shortened(int inner_order) {
    return inner_order == GHSVD_INNER_FULL_JQR || inner_order == GHSVD_INNER_FB_JQR ||
           inner_multilevel(inner_order);
}

// Blocked and FP32 stages (blocked.hip).
void set_block_geometry(PencilDev &d, int w);
size_t blocked_bytes(int mr, int n, int pr, int w, int mixed);
void carve_blocked(Carver &c, int mr, int n, int pr, int w, int mixed, PencilDev &d);
int to_fp32(const BatchCtx &c, hipStream_t s);
int fp32_handoff(const BatchCtx &c, hipStream_t s);

// Outputs (post.hip): lambda, X for one pencil; flags in small[2].
int postprocess(const PencilDev &P, int sort, hipStream_t s);

}  // namespace ghsvd
