// solver.hpp -- per-pencil plan and workspace of the solver.
#pragma once

#include "hz_common.hpp"
#include "reduce.hpp"
#include "sweep.hpp"

namespace ghsvd {

struct Plan {
    int m, n, p;    // input sizes
    int reduce;     // run the one-time reduction
    int mr, pr;     // rows of F and G as swept
    long ldft, ldgt;  // tall scratch copies
    long ldf, ldg, ldz;
    int N;          // n rounded up to even
    int mixed;      // FP32 warm-up stage
    int blocked;    // Level-2 blocked FP64 stage
};

struct BlockedWs;

struct PencilWs {
    double2 *Ft, *Gt;
    JqrBufs jq;
    double2 *qv;
    double *qcoef;
    int8_t *Jw;
    int *rowmap, *perm;
    double2 *Fw, *Gw, *Zw;
    SweepState *st;
    unsigned long long *slot_cnt;
    double *lam_tmp, *scale;
    int *rank;
    int *small;  // [0] input flags, [1] nplus, [2] output flags
    double *gnorm2;
    float2 *F32, *G32, *Z32;
    // blocked variant scratch
    void *blk;
    size_t blk_bytes;
};

Plan make_plan(int m, int n, int p, const ghsvd_options &o);
PencilWs carve(Carver &c, const Plan &pl);
size_t plan_bytes(const Plan &pl);
SweepArgs sweep_args(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o, int fp32);
int prepare_pencil(const Plan &pl, const PencilWs &w, const double2 *F, long ldf, const int8_t *J,
                   const double2 *G, long ldg, hipStream_t s, int *n2x2);
int solve_one(const Plan &pl, const PencilWs &w, const double2 *F, long ldf, const int8_t *J,
              const double2 *G, long ldg, double *lambda, double2 *X, long ldx,
              const ghsvd_options &o, ghsvd_info &info, hipStream_t s);

// Blocked variant and FP32 warm-up (blocked.hip).
void carve_blocked(Carver &c, const Plan &pl, PencilWs &w);
int run_fp32_stage(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                   ghsvd_info &info, hipStream_t s);
int run_blocked_fp64(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                     ghsvd_info &info, hipStream_t s);

}  // namespace ghsvd
