// pair_sweep.hip -- the pointwise pivot-pair kernel and the sweep-stage driver.
//
// One workgroup per pivot pair of a round-robin step (Section 6.3: the pairs
// of a step are disjoint, so they run concurrently), for every pencil of the
// batch in the same launch.  A workgroup reads its two columns of F and G
// once (coalesced: consecutive lanes read consecutive rows of a column-major
// matrix), forms the six entries of (6.1) with the split signature
// J = diag(I, -I) (Section 4.5.1 run-length form with one negative block),
// reduces them over the wavefronts and the workgroup in a fixed order,
// computes the FP64 2x2 step of Section 6.1 (every wavefront redundantly, so
// no broadcast is needed), and applies Z' to the columns still held in
// registers, then to the two columns of Z.
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>

#include "hz_step.hpp"
#include "sweep.hpp"

namespace ghsvd {

template <typename T>
struct Cplx;
template <>
struct Cplx<double> {
    using type = double2;
};
template <>
struct Cplx<float> {
    using type = float2;
};

template <typename C2>
__device__ __forceinline__ C2 upd(C2 xp, C2 xq, C2 a, C2 b) {
    // xp * a + xq * b (complex)
    C2 r;
    r.x = xp.x * a.x - xp.y * a.y + xq.x * b.x - xq.y * b.y;
    r.y = xp.x * a.y + xp.y * a.x + xq.x * b.y + xq.y * b.x;
    return r;
}

template <typename T>
__device__ __forceinline__ typename Cplx<T>::type cvt(double2 z) {
    typename Cplx<T>::type r;
    r.x = (T)z.x;
    r.y = (T)z.y;
    return r;
}

// Accumulates J-weighted (or plain) Gram entries of a column pair.
template <typename T, typename C2>
__device__ __forceinline__ void acc_pair(C2 xp, C2 xq, T sg, T &aa, T &bb, T &cr, T &ci) {
    aa += sg * (xp.x * xp.x + xp.y * xp.y);
    bb += sg * (xq.x * xq.x + xq.y * xq.y);
    // conj(xp) * xq
    cr += sg * (xp.x * xq.x + xp.y * xq.y);
    ci += sg * (xp.x * xq.y - xp.y * xq.x);
}

// One pivot pair (p, q) of pencil P: dots, 2x2 step, column updates.
template <typename T, int NT, int R>
__device__ __forceinline__ void pair_body(const PencilDev &P, int p, int q, int slot, int crit) {
    using C2 = typename Cplx<T>::type;
    constexpr bool F32 = sizeof(T) == 4;
    const int tid = threadIdx.x;
    const GPtr<C2> F(reinterpret_cast<C2 *>(F32 ? (void *)P.F32 : (void *)P.Fw));
    const GPtr<C2> G(reinterpret_cast<C2 *>(F32 ? (void *)P.G32 : (void *)P.Gw));
    const GPtr<C2> Z(reinterpret_cast<C2 *>(F32 ? (void *)P.Z32 : (void *)P.Zw));
    const GPtr<C2> Fp = F + (long)p * P.ldf, Fq = F + (long)q * P.ldf;
    const GPtr<C2> Gp = G + (long)p * P.ldg, Gq = G + (long)q * P.ldg;
    const GPtr<C2> Zp_ = Z + (long)p * P.ldz, Zq = Z + (long)q * P.ldz;
    const int m = P.mr, pr = P.pr, nplus = P.small[1], n = P.n;

    constexpr int RR = R > 0 ? R : 1;
    C2 fp[RR], fq[RR], gp[RR], gq[RR];
    T a = 0, b = 0, cr = 0, ci = 0, sa = 0, sb = 0, sr = 0, si = 0;
    if constexpr (R > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < m) {
                fp[r] = Fp.ld(i);
                fq[r] = Fq.ld(i);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < pr) {
                gp[r] = Gp.ld(i);
                gq[r] = Gq.ld(i);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < m) acc_pair<T, C2>(fp[r], fq[r], i < nplus ? T(1) : T(-1), a, b, cr, ci);
            if (i < pr) acc_pair<T, C2>(gp[r], gq[r], T(1), sa, sb, sr, si);
        }
    } else {
        for (int i = tid; i < m; i += NT)
            acc_pair<T, C2>(Fp.ld(i), Fq.ld(i), i < nplus ? T(1) : T(-1), a, b, cr, ci);
        for (int i = tid; i < pr; i += NT) acc_pair<T, C2>(Gp.ld(i), Gq.ld(i), T(1), sa, sb, sr, si);
    }

    __shared__ double red[8 * (NT / kWave)];
    double v[8] = {(double)a, (double)b, (double)cr, (double)ci,
                   (double)sa, (double)sb, (double)sr, (double)si};
    block_sum<8>(v, red);

    const double tol = (F32 ? 0x1p-23 : 0x1p-52) * sqrt((double)n);
    Zp z;
    int kind = hz_step(v[0], v[1], cmk(v[2], v[3]), v[4], v[5], cmk(v[6], v[7]), tol, crit, z,
                       F32 ? 1 : 0);
    // FP32 stage: a pair that looks dependent in FP32 is left to the FP64 sweeps;
    // the inner level of a shortened block pivot leaves it to later block sweeps.
    if ((F32 || P.skip_rank) && kind == GHSVD_ERANK) kind = kSkip;
    if (tid == 0) {
        unsigned long long *c = P.slot_cnt + 3 * slot;
        c[0] += 1ull;
        c[1] += (kind > 0) ? 1ull : 0ull;
        c[2] += (kind == kBig) ? 1ull : 0ull;
        if (kind < 0) atomicCAS(&P.st->err, 0, kind);
    }
    if (kind <= 0) return;

    const C2 z11 = cvt<T>(z.z11), z21 = cvt<T>(z.z21), z12 = cvt<T>(z.z12), z22 = cvt<T>(z.z22);
    if constexpr (R > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < m) {
                Fp.st(i, upd(fp[r], fq[r], z11, z21));
                Fq.st(i, upd(fp[r], fq[r], z12, z22));
            }
            if (i < pr) {
                Gp.st(i, upd(gp[r], gq[r], z11, z21));
                Gq.st(i, upd(gp[r], gq[r], z12, z22));
            }
        }
    } else {
        for (int i = tid; i < m; i += NT) {
            const C2 xp = Fp.ld(i), xq = Fq.ld(i);
            Fp.st(i, upd(xp, xq, z11, z21));
            Fq.st(i, upd(xp, xq, z12, z22));
        }
        for (int i = tid; i < pr; i += NT) {
            const C2 xp = Gp.ld(i), xq = Gq.ld(i);
            Gp.st(i, upd(xp, xq, z11, z21));
            Gq.st(i, upd(xp, xq, z12, z22));
        }
    }
    for (int i = tid; i < n; i += NT) {
        const C2 xp = Zp_.ld(i), xq = Zq.ld(i);
        Zp_.st(i, upd(xp, xq, z11, z21));
        Zq.st(i, upd(xp, xq, z12, z22));
    }
}

template <typename T, int NT, int R>
__global__ __launch_bounds__(NT) void k_pair(const PencilDev *PD, const int *pre, const int *flag,
                                             int B, int crit, int step) {
    const int k = find_pencil(pre, B, blockIdx.x);
    const PencilDev P = PD[k];
    if (step >= P.N - 1 || flag[k]) return;  // surplus step of a smaller pencil, or finished
    const int slot = pencil_local(pre, k, blockIdx.x);
    int p, q;
    rr_pair(P.N, step, slot, p, q);
    if (q < P.n) pair_body<T, NT, R>(P, p, q, slot, crit);  // else: bye slot of an odd order
}

__global__ void k_reset_states(const PencilDev *PD, int *flag, const int *presolved, int B,
                               int max_sweeps, int noise_floor, int blocked, int stop_all) {
    const int k = blockIdx.x;
    if (k >= B) return;
    const PencilDev P = PD[k];
    SweepState *st = P.st;
    unsigned long long *cnt = blocked ? P.bcnt : P.slot_cnt;
    const int nc = blocked ? P.nbp : P.nslots;
    for (int s = threadIdx.x; s < 3 * nc; s += blockDim.x) cnt[s] = 0ull;
    if (threadIdx.x == 0) {
        const int skip = (blocked ? (P.n < 4 || P.nb < 2) : 0) || (presolved && presolved[k]);
        st->done = skip;
        flag[k] = skip;
        st->converged = skip;
        st->sweeps = 0;
        st->err = 0;
        st->max_sweeps = max_sweeps;
        st->noise_floor = noise_floor;
        st->stop_all = stop_all;
    }
}

// End of a round, one workgroup per pencil still running: sums the per-slot
// counters of the sweep just finished in a fixed order, clears them, records
// them, and applies the stopping rules (Section 6.1.7: no big transformation
// in the sweep; Algorithm 2: the sweep cap).  The FP32 stage also stops at
// the point where its sweeps stop paying: a sweep with at most one big
// transformation per 8 visited pairs.  Later FP32 sweeps barely shorten the
// FP64 finish (an indefinite J amplifies FP32 rounding in the J-Grams beyond
// the criterion's threshold, so the FP32 big count settles well above zero),
// while each costs about two thirds of an FP64 sweep.
__global__ __launch_bounds__(256) void k_end_round(const PencilDev *PD, int *flag, int B,
                                                   int blocked) {
    __shared__ double red[3 * 256 / kWave];
    const PencilDev P = PD[blockIdx.x];
    SweepState *st = P.st;
    if (st->done) return;
    unsigned long long *cnt = blocked ? P.bcnt : P.slot_cnt;
    const int nc = blocked ? P.nbp : P.nslots;
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nc; k += blockDim.x) {
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
        } else if (v[st->stop_all ? 1 : 2] == 0.0) {
            st->done = 1;
            st->converged = 1;
        } else if (st->noise_floor && v[2] * 8.0 <= v[0]) {
            st->done = 1;
        } else if (sw + 1 >= st->max_sweeps) {
            st->done = 1;
        }
        flag[blockIdx.x] = st->done;
    }
}


// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
using PairFn = void (*)(const PencilDev *, const int *, const int *, int, int, int);

template <typename T>
static PairFn pick(int nt, int r) {
#define GHSVD_R(NT_)                                  \
    switch (r) {                                      \
        case 0: return k_pair<T, NT_, 0>;             \
        case 1: return k_pair<T, NT_, 1>;             \
        case 2: return k_pair<T, NT_, 2>;             \
        case 4: return k_pair<T, NT_, 4>;             \
        case 8: return k_pair<T, NT_, 8>;             \
        default: return nullptr;                      \
    }
    switch (nt) {
        case 64: GHSVD_R(64)
        case 128: GHSVD_R(128)
        case 256: GHSVD_R(256)
        case 512: GHSVD_R(512)
        case 1024: GHSVD_R(1024)
        default: return nullptr;
    }
#undef GHSVD_R
}

PairGeom choose_pair_geom(int rows, int waves_per_pair) {
    PairGeom g;
    int nt;
    if (waves_per_pair > 0) {
        nt = 64 * waves_per_pair;
        if (nt > 1024) nt = 1024;
    } else {
        nt = 64;
        while (nt < 1024 && nt * 4 < rows) nt *= 2;
    }
    const int per = (rows + nt - 1) / nt;
    int r = 1;
    while (r < per) r *= 2;
    g.nt = nt;
    g.r = (r <= 8) ? r : 0;
    return g;
}

int upload_batch(BatchCtx &c, hipStream_t s) {
    const int B = c.B;
    c.pre.assign(BatchCtx::kKinds * (B + 1), 0);
    c.max_n = 0;
    c.max_rows = 0;
    for (int k = 0; k < B; ++k) {
        const PencilDev &P = c.host[k];
        const int w[BatchCtx::kKinds] = {P.nslots, P.n, P.nbp * (P.kf + P.kg), P.nbp,
                                         P.nbp * P.tu, 1};
        for (int t = 0; t < BatchCtx::kKinds; ++t)
            c.pre[t * (B + 1) + k + 1] = c.pre[t * (B + 1) + k] + w[t];
        if (P.n > c.max_n) c.max_n = P.n;
        const int rows = P.mr > P.pr ? P.mr : P.pr;
        if (rows > c.max_rows) c.max_rows = rows;
    }
    GHSVD_HIP(hipMemcpyAsync(c.dev, c.host.data(), sizeof(PencilDev) * B, hipMemcpyHostToDevice, s));
    GHSVD_HIP(hipMemcpyAsync(c.pre_dev, c.pre.data(), sizeof(int) * c.pre.size(),
                             hipMemcpyHostToDevice, s));
    return GHSVD_OK;
}

void trace_stage(const char *name, int pencil, const SweepState &hs) {
    if (!std::getenv("GHSVD_TRACE")) return;
    for (int k = 0; k < hs.sweeps && k < kMaxHist; ++k)
        std::fprintf(stderr, "ghsvd %s pencil %d sweep %d: visited %llu transformed %llu big %llu\n",
                     name, pencil, k + 1, hs.hist[3 * k], hs.hist[3 * k + 1], hs.hist[3 * k + 2]);
}

// Sweep-kernel timing for measurement harnesses (see ghsvd_profile_enable):
// every `every`-th launch of each kernel kind is bracketed by two events.
namespace prof {
static std::mutex mu;
static int every = 0;
static long long launches[kProfKinds] = {};
static std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kProfKinds];
static std::vector<hipEvent_t> spare;

static hipEvent_t take_event() {
    if (!spare.empty()) {
        hipEvent_t e = spare.back();
        spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace prof

void prof_take(int kind, hipEvent_t &e0, hipEvent_t &e1) {
    e0 = e1 = nullptr;
    std::lock_guard<std::mutex> lk(prof::mu);
    if (prof::every <= 0) return;
    if (prof::launches[kind] % prof::every == 0) {
        e0 = prof::take_event();
        e1 = prof::take_event();
        if (!e0 || !e1) e0 = e1 = nullptr;
    }
    prof::launches[kind]++;
}

void prof_done(int kind, hipEvent_t e0, hipEvent_t e1) {
    if (!e0 || !e1) return;
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::pending[kind].emplace_back(e0, e1);
}

static bool prof_active() {
    std::lock_guard<std::mutex> lk(prof::mu);
    return prof::every > 0;
}

// A round captured into a graph on an internal stream (graphs cannot be
// captured on the legacy null stream the caller may pass).
struct RoundGraph {
    hipStream_t gs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    ~RoundGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (gs) (void)hipStreamDestroy(gs);
        if (ev) (void)hipEventDestroy(ev);
    }
};

static int enqueue_round(const BatchCtx &c, StepFn one_step, const void *arg, int steps,
                         int blocked, hipStream_t s) {
    for (int i = 0; i < steps; ++i) {
        const int rc = one_step(c, arg, i, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_end_round, dim3(c.B), dim3(256), 0, s, c.dev, c.flag_dev, c.B, blocked);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// Captures one round on rg.gs; false (and no graph) when any part fails.
static bool capture_round(const BatchCtx &c, StepFn one_step, const void *arg, int steps,
                          int blocked, RoundGraph &rg) {
    if (hipStreamCreateWithFlags(&rg.gs, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&rg.ev, hipEventDisableTiming) != hipSuccess) return false;
    if (hipStreamBeginCapture(rg.gs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    const int rc = enqueue_round(c, one_step, arg, steps, blocked, rg.gs);
    const bool ended = hipStreamEndCapture(rg.gs, &rg.graph) == hipSuccess;
    if (rc != GHSVD_OK || !ended) return false;
    return hipGraphInstantiate(&rg.exec, rg.graph, nullptr, nullptr, 0) == hipSuccess;
}

int drive_stage(const BatchCtx &c, int max_sweeps, int noise_floor, int blocked, StepFn one_step,
                const void *arg, int steps_per_round, const char *name, hipStream_t s,
                std::vector<SweepResult> &res, const std::vector<int> *presolved) {
    const int B = c.B;
    res.assign(B, SweepResult{GHSVD_OK, 0, 0, 0, 0, 0});
    RoundGraph rg;
    if (!c.plain && !prof_active() && !std::getenv("GHSVD_NO_GRAPH") &&
        !capture_round(c, one_step, arg, steps_per_round, blocked, rg)) {
        (void)hipGetLastError();
        if (rg.exec) (void)hipGraphExecDestroy(rg.exec);
        if (rg.graph) (void)hipGraphDestroy(rg.graph);
        rg.exec = nullptr;
        rg.graph = nullptr;
    }
    // The stage runs on the graph's stream after the caller's prior work.
    hipStream_t ss = s;
    if (rg.exec) {
        GHSVD_HIP(hipEventRecord(rg.ev, s));
        GHSVD_HIP(hipStreamWaitEvent(rg.gs, rg.ev, 0));
        ss = rg.gs;
    }
    const int *pre_dev = nullptr;
    if (presolved) {
        GHSVD_HIP(hipMemcpyAsync(c.done_dev, presolved->data(), sizeof(int) * B,
                                 hipMemcpyHostToDevice, ss));
        pre_dev = c.done_dev;
    }
    hipLaunchKernelGGL(k_reset_states, dim3(B), dim3(256), 0, ss, c.dev, c.flag_dev, pre_dev, B,
                       max_sweeps, noise_floor, blocked, c.stop_all);
    GHSVD_HIP(hipGetLastError());
    std::vector<int> done(B, 0);
    const bool trace = std::getenv("GHSVD_TRACE") != nullptr;
    bool all_pre = presolved != nullptr;
    for (int k = 0; k < B && all_pre; ++k) all_pre = (*presolved)[k] != 0;
    for (int round = 0; round < max_sweeps && !all_pre; ++round) {
        if (rg.exec) {
            GHSVD_HIP(hipGraphLaunch(rg.exec, ss));
        } else {
            const int rc = enqueue_round(c, one_step, arg, steps_per_round, blocked, ss);
            if (rc) return rc;
        }
        GHSVD_HIP(hipMemcpyAsync(done.data(), c.flag_dev, sizeof(int) * B, hipMemcpyDeviceToHost, ss));
        GHSVD_HIP(hipStreamSynchronize(ss));
        bool all = true;
        int ndone = 0;
        for (int k = 0; k < B; ++k) {
            all = all && done[k];
            ndone += done[k] != 0;
        }
        if (trace)
            std::fprintf(stderr, "ghsvd %s round %d: %d of %d pencils done\n", name, round + 1,
                         ndone, B);
        if (all) break;
    }
    int worst = GHSVD_OK;
    for (int k = 0; k < B; ++k) {
        SweepState hs;
        GHSVD_HIP(hipMemcpyAsync(&hs, c.host[k].st, sizeof(SweepState), hipMemcpyDeviceToHost, ss));
        GHSVD_HIP(hipStreamSynchronize(ss));
        trace_stage(name, k, hs);
        SweepResult &r = res[k];
        r.sweeps = hs.sweeps;
        r.converged = hs.converged;
        for (int q = 0; q < hs.sweeps && q < kMaxHist; ++q) {
            r.visited += (long long)hs.hist[3 * q + 0];
            r.transformed += (long long)hs.hist[3 * q + 1];
            r.big += (long long)hs.hist[3 * q + 2];
        }
        r.status = hs.err ? hs.err : (hs.converged ? GHSVD_OK : GHSVD_NOT_CONVERGED);
        if (r.status < 0) worst = r.status;
    }
    return worst < 0 ? worst : GHSVD_OK;
}

struct PointwiseArg {
    PairFn fn;
    PairGeom g;
    int crit;
    int fp32;
};

static int pointwise_step(const BatchCtx &c, const void *arg, int step, hipStream_t s) {
    const PointwiseArg *a = static_cast<const PointwiseArg *>(arg);
    const int kind = a->fp32 ? kProfPair32 : kProfPair64;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!c.plain) prof_take(kind, e0, e1);
    launch_ev(a->fn, dim3(c.total(BatchCtx::kSlots)), dim3(a->g.nt), 0, s, e0, e1, c.dev,
              c.pre_of(BatchCtx::kSlots), c.flag_dev, c.B, a->crit, step);
    prof_done(kind, e0, e1);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

int run_pointwise_stage(const BatchCtx &c, int fp32, int max_sweeps, int crit, PairGeom g,
                        hipStream_t s, std::vector<SweepResult> &res,
                        const std::vector<int> *presolved) {
    PointwiseArg a{fp32 ? pick<float>(g.nt, g.r) : pick<double>(g.nt, g.r), g, crit, fp32};
    if (!a.fn) return GHSVD_EINVAL;
    int steps = 1;
    for (const PencilDev &P : c.host) steps = P.N - 1 > steps ? P.N - 1 : steps;
    return drive_stage(c, max_sweeps, fp32, 0, pointwise_step, &a, steps,
                       fp32 ? "pointwise-fp32" : "pointwise-fp64", s, res, presolved);
}

// ---------------------------------------------------------------------------
// Batched 2x2 step (component entry point).
// ---------------------------------------------------------------------------
__global__ void k_pair_params(int count, const double *a, const double *b, const double2 *c,
                              const double *sa, const double *sb, const double2 *sc, double tol,
                              int crit, double2 *Z, int *kind) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    Zp z;
    kind[i] = hz_step(a[i], b[i], c[i], sa[i], sb[i], sc[i], tol, crit, z);
    Z[4 * i + 0] = z.z11;
    Z[4 * i + 1] = z.z21;
    Z[4 * i + 2] = z.z12;
    Z[4 * i + 3] = z.z22;
}

}  // namespace ghsvd

using namespace ghsvd;

extern "C" int ghsvd_pair_params(int count, const double *a, const double *b, const double *c,
                                 const double *sa, const double *sb, const double *sc,
                                 double tol, int crit_literal, double *Z, int *kind,
                                 void *stream) {
    if (count < 0) return GHSVD_EINVAL;
    if (count == 0) return GHSVD_OK;
    if (!a || !b || !c || !sa || !sb || !sc || !Z || !kind) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_pair_params, dim3((count + 255) / 256), dim3(256), 0, s, count, a, b,
                       reinterpret_cast<const double2 *>(c), sa, sb,
                       reinterpret_cast<const double2 *>(sc), tol, crit_literal,
                       reinterpret_cast<double2 *>(Z), kind);
    GHSVD_HIP(hipGetLastError());
    GHSVD_HIP(hipStreamSynchronize(s));
    return GHSVD_OK;
}

extern "C" int ghsvd_round_robin(int n, int *p_out, int *q_out) {
    if (n < 1 || !p_out || !q_out) return -1;
    const int N = n + (n & 1);
    const int slots = N / 2;
    if (N < 2) return 0;
    for (int s = 0; s < N - 1; ++s)
        for (int k = 0; k < slots; ++k) {
            int p, q;
            rr_pair(N, s, k, p, q);
            if (q >= n) p = q = -1;
            p_out[s * slots + k] = p;
            q_out[s * slots + k] = q;
        }
    return N - 1;
}

extern "C" void ghsvd_profile_enable(int every) {
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::every = every > 0 ? every : 0;
    for (long long &l : prof::launches) l = 0;
}

extern "C" int ghsvd_profile_read(int kind, double *ms, long long *timed, long long *launches) {
    if (kind < 0 || kind >= kProfKinds) return GHSVD_EINVAL;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    long long nl;
    {
        std::lock_guard<std::mutex> lk(prof::mu);
        ev.swap(prof::pending[kind]);
        nl = prof::launches[kind];
        prof::launches[kind] = 0;
    }
    double tot = 0.0;
    int rc = GHSVD_OK;
    for (auto &e : ev) {
        float t = 0.0f;
        if (hipEventSynchronize(e.second) != hipSuccess ||
            hipEventElapsedTime(&t, e.first, e.second) != hipSuccess)
            rc = GHSVD_EDEVICE;
        tot += t;
    }
    {
        std::lock_guard<std::mutex> lk(prof::mu);
        for (auto &e : ev) {
            prof::spare.push_back(e.first);
            prof::spare.push_back(e.second);
        }
    }
    if (ms) *ms = tot;
    if (timed) *timed = (long long)ev.size();
    if (launches) *launches = nl;
    return rc;
}
