// solver.hip -- the C entry points.  ghsvd_solve is a batch of one pencil;
// ghsvd_solve_batched runs all pencils' reductions and sweeps together, each
// launch covering every pencil still active.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "reduce.hpp"
#include "solver.hpp"
#include "sweep.hpp"

#ifndef GHSVD_SPLIT_GROUPS
#define GHSVD_SPLIT_GROUPS 2
#endif

namespace ghsvd {

void fill_options(const ghsvd_options *opt, ghsvd_options &o) {
    ghsvd_default_options(&o);
    if (opt) o = *opt;
    if (o.max_sweeps <= 0) o.max_sweeps = kDefaultMaxSweeps;
    if (o.max_sweeps > kMaxHist) o.max_sweeps = kMaxHist;
}

Plan make_plan(int m, int n, int p, const ghsvd_options &o, int block_width) {
    Plan pl{};
    pl.m = m;
    pl.n = n;
    pl.p = p;
    pl.reduce = o.reduce && (m > n || p > n);
    pl.mr = pl.reduce ? n : m;
    pl.pr = pl.reduce ? n : p;
    pl.ldft = pad_ld(m);
    pl.ldgt = pad_ld(p);
    pl.ldf = pad_ld(pl.mr);
    pl.ldg = pad_ld(pl.pr);
    pl.ldz = pad_ld(n);
    pl.N = n + (n & 1);
    pl.mixed = (o.precision == GHSVD_MIXED);
    pl.blocked = (o.variant == GHSVD_BLOCKED);
    pl.w = block_width;
    return pl;
}

void carve_pencil(Carver &c, const Plan &pl, PencilDev &d) {
    const int n = pl.n;
    d.m = pl.m;
    d.n = n;
    d.p = pl.p;
    d.mr = pl.mr;
    d.pr = pl.pr;
    d.reduce = pl.reduce;
    d.N = pl.N;
    d.nslots = pl.N / 2;
    d.ldft = pl.ldft;
    d.ldgt = pl.ldgt;
    d.ldf = pl.ldf;
    d.ldg = pl.ldg;
    d.ldz = pl.ldz;
    d.jst = c.take<JqrState>(2);
    if (pl.reduce) {
        d.Ft = c.take<double2>((size_t)pl.ldft * n);
        d.Gt = c.take<double2>((size_t)pl.ldgt * n);
        d.jdec = c.take<JqrDecision>(1);
        d.hd = c.take<double>(n);
        d.hl = c.take<double>(n);
        d.hc = c.take<double2>(n);
        d.hi = c.take<double>(n);
        d.cpb = c.take<int>(n);
        d.rblk = c.take<double2>(2 * (size_t)n);
        d.pblk = c.take<int>(2 * (size_t)n);
        d.qdiag = c.take<double2>(n);
        d.qnrm = c.take<double>(n);
    }
    d.Jw = c.take<int8_t>(2 * (size_t)pl.m);
    d.rowmap = c.take<int>(pl.m > n ? pl.m : n);
    d.perm = c.take<int>(n);
    if (!pl.inplace) {
        d.Fw = c.take<double2>((size_t)pl.ldf * n);
        d.Gw = c.take<double2>((size_t)pl.ldg * n);
        d.Zw = c.take<double2>((size_t)pl.ldz * n);
    }
    d.st = c.take<SweepState>(1);
    d.slot_cnt = c.take<unsigned long long>(3 * (size_t)(pl.N / 2 + 1));
    d.lam_tmp = c.take<double>(n);
    d.scale = c.take<double>(n);
    d.rank = c.take<int>(n);
    d.small = c.take<int>(8);
    d.gnorm2 = c.take<double>(1 + 8 * (size_t)n);  // ||G||_F^2 and its partials
    if (pl.mixed) {
        d.F32 = c.take<float2>((size_t)pl.ldf * n);
        d.G32 = c.take<float2>((size_t)pl.ldg * n);
        d.Z32 = c.take<float2>((size_t)pl.ldz * n);
    }
    if (pl.blocked || pl.mixed) {
        carve_blocked(c, pl.mr, n, pl.pr, pl.w, pl.mixed, d);
        set_block_geometry(d, pl.w);
    } else {
        d.w = pl.w;
        d.nb = 0;
        d.nbp = 0;
    }
}

size_t pencil_bytes(const Plan &pl) {
    Carver c{nullptr, 0, (size_t)-1};
    PencilDev d{};
    carve_pencil(c, pl, d);
    return align_up(c.used, 256) + 256;
}

size_t batch_bytes(int B) {
    return align_up(sizeof(PencilDev) * B, 256) +
           align_up(sizeof(int) * BatchCtx::kKinds * (B + 1), 256) +
           align_up(sizeof(int) * 2 * kWinRows * (B + 1), 256) +
           align_up(sizeof(int) * 2 * (B + 1), 256) + align_up(sizeof(int) * (B + 1), 256) + 256;
}

void carve_batch(Carver &c, BatchCtx &bc, int B) {
    bc.dev = c.take<PencilDev>(B);
    bc.pre_dev = c.take<int>(BatchCtx::kKinds * (B + 1));
    bc.win_dev = c.take<int>(2 * kWinRows * (B + 1));
    bc.done_dev = c.take<int>(2 * (B + 1));
    bc.flag_dev = c.take<int>(B + 1);
}

__global__ void k_zero_small(const PencilDev *PD, int B) {
    const int k = blockIdx.x;
    if (k >= B) return;
    if (threadIdx.x < 8) PD[k].small[threadIdx.x] = 0;
    if (threadIdx.x == 0) PD[k].gnorm2[0] = 0.0;
}

__global__ void k_gather_small(const PencilDev *PD, int B, int idx, int *out) {
    for (int k = threadIdx.x; k < B; k += blockDim.x) out[k] = PD[k].small[idx];
}

static int gather_small(const BatchCtx &c, int idx, std::vector<int> &out, hipStream_t s) {
    out.assign(c.B, 0);
    hipLaunchKernelGGL(k_gather_small, dim3(1), dim3(256), 0, s, c.dev, c.B, idx, c.done_dev);
    GHSVD_HIP(hipGetLastError());
    GHSVD_HIP(hipMemcpyAsync(out.data(), c.done_dev, sizeof(int) * c.B, hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    return GHSVD_OK;
}

static int worst_of(int a, int b) {
    if (a < 0 || b < 0) return a < b ? a : b;
    return a > b ? a : b;
}

// Keeps only the pencils whose status is still non-negative.
static int compact(BatchCtx &c, std::vector<int> &idx, const std::vector<int> &status,
                   hipStream_t s) {
    std::vector<PencilDev> keep;
    std::vector<int> kidx;
    for (size_t k = 0; k < idx.size(); ++k)
        if (status[idx[k]] >= 0) {
            keep.push_back(c.host[k]);
            kidx.push_back(idx[k]);
        }
    if (kidx.size() == idx.size()) return GHSVD_OK;
    c.host.swap(keep);
    idx.swap(kidx);
    c.B = (int)c.host.size();
    if (c.B == 0) return GHSVD_OK;
    return upload_batch(c, s);
}

// ---------------------------------------------------------------------------
// Tuned launch parameters.  ghsvd_autotune times trial sweeps and stores the
// fastest block width and wavefronts per pair for a shape class (variant,
// precision, and the base-2 size classes of the batch, the largest order and
// the largest swept row count); solves that leave these options at 0 use the
// stored values, else fixed rules.  The cache is the library's only global
// state and is guarded by a mutex.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
    int variant, precision, bcls, ncls, rcls;
    bool operator<(const TuneKey &o) const {
        return std::tie(variant, precision, bcls, ncls, rcls) <
               std::tie(o.variant, o.precision, o.bcls, o.ncls, o.rcls);
    }
};
struct TuneVal {
    int w, wpp;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int log2_class(int x) {
    int c = 0;
    while ((1 << c) < x && c < 30) ++c;
    return c;
}

TuneKey tune_key(const std::vector<PencilIO> &io, const ghsvd_options &o) {
    int max_n = 0, max_rows = 0;
    for (const PencilIO &p : io) {
        const bool red = o.reduce && (p.m > p.n || p.p > p.n);
        const int rows = red ? p.n : std::max(p.m, p.p);
        max_n = std::max(max_n, p.n);
        max_rows = std::max(max_rows, rows);
    }
    return TuneKey{o.variant, o.precision, log2_class((int)io.size()), log2_class(max_n),
                   log2_class(max_rows)};
}
}  // namespace

// Block width and wavefronts per pair for this batch: the options when set,
// else the tuned values for the shape class, else the fixed rules.
static void resolve_launch(const std::vector<PencilIO> &io, const ghsvd_options &o, int &w,
                           int &wpp) {
    int max_n = 0;
    for (const PencilIO &p : io) max_n = std::max(max_n, p.n);
    w = o.block_width;
    wpp = o.waves_per_pair;
    if (w == 0 || wpp == 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(io, o));
        if (it != g_tune.end()) {
            if (w == 0) w = it->second.w;
            if (wpp == 0) wpp = it->second.wpp;
        }
    }
    w = pick_block_width(max_n, w);
}

// Workspace bytes: with an automatic block width the larger of the widths'
// needs, so that a later tuned choice always fits.
size_t solve_batch_bytes(const std::vector<PencilIO> &io, const ghsvd_options &o) {
    int max_n = 0;
    for (const PencilIO &p : io) max_n = p.n > max_n ? p.n : max_n;
    size_t total = batch_bytes((int)io.size());
    for (const PencilIO &p : io) {
        size_t need = 0;
        for (int w : {8, 16, 32}) {
            if (o.block_width != 0 && o.block_width != w) continue;
            need = std::max(need, pencil_bytes(make_plan(p.m, p.n, p.p, o, w)));
        }
        total += need;
    }
    if (o.variant == GHSVD_BLOCKED && inner_shortened(o.inner_order)) {
        size_t need = 0;
        for (int w : {8, 16, 32}) {
            if (o.block_width != 0 && o.block_width != w) continue;
            std::vector<Plan> pl;
            for (const PencilIO &p : io) pl.push_back(make_plan(p.m, p.n, p.p, o, w));
            need = std::max(need, short_stage_bytes(pl, w));
        }
        total += align_up(need, 256) + 256;
    }
    return total;
}

int solve_batch(const std::vector<PencilIO> &io, const ghsvd_options &o, void *work, size_t lwork,
                std::vector<ghsvd_info> &info, hipStream_t s, StageClock *clk) {
    const int B0 = (int)io.size();
    info.assign(B0, ghsvd_info{});
    std::vector<int> status(B0, GHSVD_OK);
    int w, wpp;
    resolve_launch(io, o, w, wpp);
    Carver c{reinterpret_cast<char *>(work), 0, lwork};
    BatchCtx bc;
    carve_batch(c, bc, B0);
    bc.B = B0;
    bc.host.resize(B0);
    std::vector<int> idx(B0);
    for (int k = 0; k < B0; ++k) {
        const PencilIO &p = io[k];
        const Plan pl = make_plan(p.m, p.n, p.p, o, w);
        PencilDev &d = bc.host[k];
        d = PencilDev{};
        c.used = align_up(c.used, 256);
        carve_pencil(c, pl, d);
        d.Fin = p.F;
        d.ldfin = p.ldf;
        d.Jin = p.J;
        d.Gin = p.G;
        d.ldgin = p.ldg;
        d.lambda = p.lambda;
        d.X = p.X;
        d.ldx = p.ldx;
        idx[k] = k;
        info[k].m_r = pl.mr;
        info[k].p_r = pl.pr;
    }
    if (o.variant == GHSVD_BLOCKED && inner_shortened(o.inner_order)) {
        std::vector<Plan> pl;
        for (const PencilIO &p : io) pl.push_back(make_plan(p.m, p.n, p.p, o, w));
        bc.short_cap = short_stage_bytes(pl, w);
        bc.short_buf = c.take<char>(bc.short_cap);
    }
    if (!c.ok()) return GHSVD_ENOMEM;
    int rc = upload_batch(bc, s);
    if (rc) return rc;

    // 1. input checks
    hipLaunchKernelGGL(k_zero_small, dim3(bc.B), dim3(64), 0, s, bc.dev, bc.B);
    for (const PencilDev &P : bc.host)
        if ((rc = check_inputs(P.m, P.n, P.p, P.Fin, P.ldfin, P.Jin, P.Gin, P.ldgin, P.small,
                               P.gnorm2, s)))
            return rc;
    std::vector<int> fl;
    if ((rc = gather_small(bc, 0, fl, s))) return rc;
    for (int k = 0; k < bc.B; ++k) {
        if (fl[k] & 1) status[idx[k]] = GHSVD_EINVAL;
        else if (fl[k] & 2) status[idx[k]] = GHSVD_ENONFINITE;
    }
    if ((rc = compact(bc, idx, status, s))) return rc;

    // 2. one-time reduction (batched), signature split, sweep buffers
    if (bc.B > 0) {
        std::vector<int> rst, n2;
        if ((rc = run_reduction(bc, rst, n2, s))) return rc;
        for (int k = 0; k < bc.B; ++k) {
            info[idx[k]].n2x2 = n2[k];
            if (rst[k]) status[idx[k]] = rst[k];
        }
        if ((rc = compact(bc, idx, status, s))) return rc;
    }
    for (const PencilDev &P : bc.host) {
        if (P.reduce) {
            if ((rc = jsplit_map(P.n, P.Jw, P.rowmap, P.small + 1, s))) return rc;
            if ((rc = jqr_extract(P, P.Fw, P.ldf, P.rowmap, s))) return rc;
            if ((rc = copy_cols(P.n, P.n, P.Gt, P.ldgt, P.Gw, P.ldg, P.perm, s))) return rc;
        } else {
            if ((rc = jsplit(P.m, P.n, P.Fin, P.ldfin, P.Jin, P.Fw, P.ldf, P.rowmap, P.small + 1, s)))
                return rc;
            if ((rc = copy_cols(P.p, P.n, P.Gin, P.ldgin, P.Gw, P.ldg, nullptr, s))) return rc;
        }
        if ((rc = set_identity(P.n, P.Zw, P.ldz, 0, s))) return rc;
    }
    if (bc.B > 0) {
        std::vector<int> np;
        if ((rc = gather_small(bc, 1, np, s))) return rc;
        for (int k = 0; k < bc.B; ++k) info[idx[k]].n_plus = np[k];
    }

    // 3. sweep stages: the FP32 warm-up (blocked or pointwise) with its FP64
    // hand-off when mixed; FP64 blocked sweeps for the blocked variant; then
    // FP64 pointwise sweeps for every pencil the blocked stage did not
    // finish.
    auto account = [&](const std::vector<SweepResult> &r, int fp32, int blocked) {
        for (int k = 0; k < bc.B; ++k) {
            ghsvd_info &inf = info[idx[k]];
            if (fp32) inf.sweeps_fp32 += r[k].sweeps;
            else inf.sweeps_fp64 += r[k].sweeps;
            if (blocked) inf.sweeps_blocked += r[k].sweeps;
            inf.pairs_visited += r[k].visited;
            inf.pairs_transformed += r[k].transformed;
            inf.pairs_big += r[k].big;
            if (!fp32 && !blocked) {
                inf.pw_visited += r[k].visited;
                inf.pw_transformed += r[k].transformed;
            }
        }
    };
    std::vector<SweepResult> res;
    std::vector<int> presolved;
    if (bc.B > 0 && o.precision == GHSVD_MIXED) {
        if ((rc = to_fp32(bc, s))) return rc;
        const int blk = o.variant == GHSVD_BLOCKED;
        if (blk) rc = run_blocked_stage(bc, 1, o.max_sweeps, o.crit_literal, o.inner_order, s, res);
        else rc = run_pointwise_stage(bc, 1, o.max_sweeps, o.crit_literal,
                                      choose_pair_geom(bc.max_rows, wpp), s, res);
        if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) return rc;
        account(res, 1, blk);
        if ((rc = fp32_handoff(bc, s))) return rc;
    }
    // events around the FP64 stages when the tuner times them
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    if (clk)
        for (int i = 0; i < 4; ++i) GHSVD_HIP(hipEventCreate(&ev[i]));
    if (bc.B > 0 && o.variant == GHSVD_BLOCKED) {
        if (clk) GHSVD_HIP(hipEventRecord(ev[0], s));
        rc = run_blocked_stage(bc, 0, o.max_sweeps, o.crit_literal, o.inner_order, s, res);
        if (clk) {
            GHSVD_HIP(hipEventRecord(ev[1], s));
            GHSVD_HIP(hipEventSynchronize(ev[1]));
            GHSVD_HIP(hipEventElapsedTime(&clk->blocked_ms, ev[0], ev[1]));
        }
        if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) return rc;
        account(res, 0, 1);
        for (int k = 0; k < bc.B; ++k)
            if (res[k].status < 0) status[idx[k]] = res[k].status;
        // A blocked sweep visits every column pair, so one without a big
        // transformation meets the stopping rule (Section 6.1.7): those
        // pencils are done; the rest (sweep cap, or no blocked sweep) go on
        // with pointwise FP64 sweeps.
        // (compaction keeps the pencils with status >= 0, in order)
        presolved.clear();
        for (int k = 0; k < bc.B; ++k)
            if (status[idx[k]] >= 0)
                presolved.push_back(res[k].status == GHSVD_OK && res[k].converged &&
                                    res[k].sweeps > 0);
        if ((rc = compact(bc, idx, status, s))) return rc;
    }
    if (bc.B > 0) {
        if (clk) GHSVD_HIP(hipEventRecord(ev[2], s));
        rc = run_pointwise_stage(bc, 0, o.max_sweeps, o.crit_literal,
                                 choose_pair_geom(bc.max_rows, wpp), s, res,
                                 presolved.empty() ? nullptr : &presolved);
        if (clk) {
            GHSVD_HIP(hipEventRecord(ev[3], s));
            GHSVD_HIP(hipEventSynchronize(ev[3]));
            GHSVD_HIP(hipEventElapsedTime(&clk->pointwise_ms, ev[2], ev[3]));
        }
        if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) return rc;
        account(res, 0, 0);
        for (int k = 0; k < bc.B; ++k) status[idx[k]] = res[k].status;
        if ((rc = compact(bc, idx, status, s))) return rc;
    }

    // 4. outputs
    if (clk) return GHSVD_OK;  // timing trial: no outputs
    for (const PencilDev &P : bc.host)
        if ((rc = postprocess(P, o.sort, s))) return rc;
    if (bc.B > 0) {
        std::vector<int> of;
        if ((rc = gather_small(bc, 2, of, s))) return rc;
        for (int k = 0; k < bc.B; ++k) {
            if (of[k] & 2) status[idx[k]] = GHSVD_ENONFINITE;
            else if (of[k] & 1) status[idx[k]] = GHSVD_ERANK;
        }
    }
    int worst = GHSVD_OK;
    for (int k = 0; k < B0; ++k) {
        info[k].status = status[k];
        worst = worst_of(worst, status[k]);
    }
    return worst;
}

// A one-pencil batch whose sweep buffers are the caller's (component entry
// points).  Owns its scratch allocation.
struct OwnedBatch {
    BatchCtx bc;
    void *buf = nullptr;
    ~OwnedBatch() {
        if (buf) (void)hipFree(buf);
    }
};

// Plan of a one-pencil batch swept in place on the caller's F, G, Z.
static Plan inplace_plan(int m, int n, int p, int blocked, int w) {
    ghsvd_options o;
    fill_options(nullptr, o);
    o.reduce = 0;
    o.variant = blocked ? GHSVD_BLOCKED : GHSVD_POINTWISE;
    Plan pl = make_plan(m, n, p, o, w);
    pl.inplace = 1;
    return pl;
}

static size_t inplace_bytes(int m, int n, int p, int blocked, int w) {
    return batch_bytes(1) + pencil_bytes(inplace_plan(m, n, p, blocked, w));
}

// The shortened blocked stage's region of a one-pencil in-place batch.
static size_t inplace_short_bytes(int m, int n, int p, int w) {
    return align_up(short_stage_bytes({inplace_plan(m, n, p, 1, w)}, w), 256) + 256;
}

// Carves a one-pencil in-place batch from buf (cap bytes, 256-byte aligned)
// and uploads its descriptor.
static int inplace_batch_at(BatchCtx &bc, void *buf, size_t cap, int m, int n, int p, double *F,
                            int ldf, double *G, int ldg, double *Z, int ldz, int blocked, int w,
                            hipStream_t s) {
    const Plan pl = inplace_plan(m, n, p, blocked, w);
    Carver c{reinterpret_cast<char *>(buf), 0, cap};
    carve_batch(c, bc, 1);
    bc.B = 1;
    bc.host.resize(1);
    PencilDev &d = bc.host[0];
    d = PencilDev{};
    c.used = align_up(c.used, 256);
    carve_pencil(c, pl, d);
    if (!c.ok()) return GHSVD_ENOMEM;
    d.Fw = reinterpret_cast<double2 *>(F);
    d.ldf = ldf;
    d.Gw = reinterpret_cast<double2 *>(G);
    d.ldg = ldg;
    d.Zw = reinterpret_cast<double2 *>(Z);
    d.ldz = ldz;
    return upload_batch(bc, s);
}

static int make_inplace_batch(OwnedBatch &ob, int m, int n, int p, double *F, int ldf, double *G,
                              int ldg, double *Z, int ldz, int blocked, int w, hipStream_t s,
                              int shortened = 0) {
    const size_t base = align_up(inplace_bytes(m, n, p, blocked, w), 256);
    const size_t extra = shortened ? inplace_short_bytes(m, n, p, w) : 0;
    GHSVD_HIP(hipMalloc(&ob.buf, base + extra));
    const int rc = inplace_batch_at(ob.bc, ob.buf, base, m, n, p, F, ldf, G, ldg, Z, ldz, blocked,
                                    w, s);
    if (shortened) {
        ob.bc.short_buf = reinterpret_cast<char *>(ob.buf) + base;
        ob.bc.short_cap = extra;
    }
    return rc;
}

__global__ void k_set_nplus(const PencilDev *PD, int nplus) { PD[0].small[1] = nplus; }

static int copy_counters(const BatchCtx &bc, int nsweeps, long long *counters, int *sweeps_done,
                         hipStream_t s) {
    SweepState hs;
    GHSVD_HIP(hipMemcpyAsync(&hs, bc.host[0].st, sizeof(SweepState), hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    if (counters)
        for (int k = 0; k < nsweeps; ++k)
            for (int j = 0; j < 3; ++j)
                counters[3 * k + j] = k < hs.sweeps ? (long long)hs.hist[3 * k + j] : 0;
    if (sweeps_done) *sweeps_done = hs.sweeps;
    return GHSVD_OK;
}

}  // namespace ghsvd

using namespace ghsvd;

extern "C" void ghsvd_default_options(ghsvd_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = GHSVD_FP64;
    opt->variant = GHSVD_POINTWISE;
    opt->reduce = 1;
    opt->block_width = 0;
    opt->waves_per_pair = 0;
    opt->max_sweeps = kDefaultMaxSweeps;
    opt->sort = 1;
    opt->crit_literal = 0;
    opt->inner_order = GHSVD_INNER_CROSS;
}

extern "C" const char *ghsvd_status_string(int status) {
    switch (status) {
        case GHSVD_OK: return "ok";
        case GHSVD_NOT_CONVERGED: return "not converged (sweep cap reached)";
        case GHSVD_EINVAL: return "invalid argument";
        case GHSVD_ERANK: return "G numerically rank deficient";
        case GHSVD_ENONFINITE: return "non-finite value";
        case GHSVD_ENOMEM: return "workspace too small";
        case GHSVD_EDEVICE: return "HIP runtime error";
        default: return "unknown status";
    }
}

static bool valid_sizes(int m, int n, int p) { return n >= 1 && m >= n && p >= n; }

static bool valid_options(const ghsvd_options &o) {
    return (o.precision == GHSVD_FP64 || o.precision == GHSVD_MIXED) &&
           (o.variant == GHSVD_POINTWISE || o.variant == GHSVD_BLOCKED) &&
           (o.block_width == 0 || o.block_width == 8 || o.block_width == 16 ||
            o.block_width == 32) &&
           o.waves_per_pair >= 0 && o.waves_per_pair <= 16 &&
           (o.inner_order == GHSVD_INNER_FULL || o.inner_order == GHSVD_INNER_CROSS ||
            o.inner_order == GHSVD_INNER_FB || inner_shortened(o.inner_order));
}

extern "C" size_t ghsvd_workspace_size(int m, int n, int p, const ghsvd_options *opt) {
    if (!valid_sizes(m, n, p)) return 0;
    ghsvd_options o;
    fill_options(opt, o);
    std::vector<PencilIO> io(1);
    io[0] = PencilIO{m, n, p, nullptr, m, nullptr, nullptr, p, nullptr, nullptr, n};
    return solve_batch_bytes(io, o);
}

static size_t batch_need(const std::vector<PencilIO> &io, const ghsvd_options &o);

extern "C" size_t ghsvd_workspace_size_batched(int batch, const int *m, const int *n, const int *p,
                                               const ghsvd_options *opt) {
    if (batch < 1 || !m || !n || !p) return 0;
    ghsvd_options o;
    fill_options(opt, o);
    std::vector<PencilIO> io(batch);
    for (int k = 0; k < batch; ++k) {
        if (!valid_sizes(m[k], n[k], p[k])) return 0;
        io[k] = PencilIO{m[k], n[k], p[k], nullptr, m[k], nullptr, nullptr, p[k], nullptr, nullptr, n[k]};
    }
    return batch_need(io, o);
}

// A batch of at least kSplitPencils pencils runs as kSplitGroups groups of
// about equal work (n^3, longest first), each on its own stream driven by
// its own host thread: the groups' kernels then overlap on the GPU, one
// group's latency-bound launches (reduction column steps, inner sweeps)
// beside another's bandwidth-bound ones.  No computation crosses pencils,
// so every pencil's result is the same as in a single solve.
constexpr int kSplitPencils = 16;
constexpr int kSplitGroups = GHSVD_SPLIT_GROUPS;

static bool split_batch(const std::vector<PencilIO> &io, std::vector<std::vector<int>> &g) {
    g.clear();
    if ((int)io.size() < kSplitPencils || kSplitGroups < 2) return false;
    std::vector<int> ord(io.size());
    for (size_t k = 0; k < io.size(); ++k) ord[k] = (int)k;
    auto work = [&](int k) { return (double)io[k].n * io[k].n * io[k].n; };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work(a) > work(b); });
    g.assign(kSplitGroups, {});
    std::vector<double> w(kSplitGroups, 0.0);
    for (int k : ord) {
        int best = 0;
        for (int i = 1; i < kSplitGroups; ++i)
            if (w[i] < w[best]) best = i;
        g[best].push_back(k);
        w[best] += work(k);
    }
    for (auto &x : g) std::sort(x.begin(), x.end());
    return true;
}

static std::vector<PencilIO> pick(const std::vector<PencilIO> &io, const std::vector<int> &g) {
    std::vector<PencilIO> r;
    for (int k : g) r.push_back(io[k]);
    return r;
}

// Workspace of a batch as run_with_workspace runs it.
static size_t batch_need(const std::vector<PencilIO> &io, const ghsvd_options &o) {
    std::vector<std::vector<int>> g;
    if (!split_batch(io, g)) return solve_batch_bytes(io, o);
    size_t total = 0;
    for (const auto &x : g) total += align_up(solve_batch_bytes(pick(io, x), o), 256);
    return total;
}

// The groups of a split batch, each on its own stream and host thread.
static int solve_split(const std::vector<PencilIO> &io, const std::vector<std::vector<int>> &g,
                       const ghsvd_options &o, void *work, std::vector<ghsvd_info> &info,
                       hipStream_t s) {
    const int G = (int)g.size();
    std::vector<std::vector<PencilIO>> iog(G);
    std::vector<size_t> off(G + 1, 0);
    for (int i = 0; i < G; ++i) {
        iog[i] = pick(io, g[i]);
        off[i + 1] = off[i] + align_up(solve_batch_bytes(iog[i], o), 256);
    }
    std::vector<hipStream_t> st(G, nullptr);
    std::vector<hipEvent_t> ev(G + 1, nullptr);
    struct Guard {
        std::vector<hipStream_t> &st;
        std::vector<hipEvent_t> &ev;
        ~Guard() {
            for (hipStream_t x : st)
                if (x) (void)hipStreamDestroy(x);
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
        }
    } guard{st, ev};
    for (int i = 0; i < G; ++i) GHSVD_HIP(hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking));
    for (int i = 0; i <= G; ++i) GHSVD_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    // every group starts after the caller's prior work on s
    GHSVD_HIP(hipEventRecord(ev[G], s));
    for (int i = 0; i < G; ++i) GHSVD_HIP(hipStreamWaitEvent(st[i], ev[G], 0));
    std::vector<std::vector<ghsvd_info>> inf(G);
    std::vector<int> rc(G, GHSVD_OK);
    char *w = reinterpret_cast<char *>(work);
    std::vector<std::thread> th;
    for (int i = 1; i < G; ++i)
        th.emplace_back([&, i] {
            rc[i] = solve_batch(iog[i], o, w + off[i], off[i + 1] - off[i], inf[i], st[i]);
        });
    rc[0] = solve_batch(iog[0], o, w, off[1], inf[0], st[0]);
    for (auto &t : th) t.join();
    // s continues after every group
    for (int i = 0; i < G; ++i) {
        GHSVD_HIP(hipEventRecord(ev[i], st[i]));
        GHSVD_HIP(hipStreamWaitEvent(s, ev[i], 0));
    }
    GHSVD_HIP(hipStreamSynchronize(s));
    info.assign(io.size(), ghsvd_info{});
    int worst = GHSVD_OK;
    for (int i = 0; i < G; ++i) {
        for (size_t k = 0; k < g[i].size(); ++k) {
            if (k < inf[i].size()) info[g[i][k]] = inf[i][k];
            else info[g[i][k]].status = rc[i] < 0 ? rc[i] : GHSVD_EDEVICE;
        }
        worst = worst_of(worst, rc[i]);
    }
    return worst;
}

static int run_with_workspace(const std::vector<PencilIO> &io, const ghsvd_options &o, void *work,
                              size_t lwork, std::vector<ghsvd_info> &info, hipStream_t s) {
    const size_t need = batch_need(io, o);
    void *own = nullptr;
    if (!work) {
        if (hipMalloc(&own, need) != hipSuccess) return GHSVD_EDEVICE;
        work = own;
        lwork = need;
    }
    int rc;
    if (lwork < need) {
        rc = GHSVD_ENOMEM;
        info.assign(io.size(), ghsvd_info{});
        for (auto &i : info) i.status = rc;
    } else {
        std::vector<std::vector<int>> g;
        rc = split_batch(io, g) ? solve_split(io, g, o, work, info, s)
                                : solve_batch(io, o, work, lwork, info, s);
        if (rc == GHSVD_EDEVICE || rc == GHSVD_ENOMEM)
            for (auto &i : info)
                if (i.status >= 0) i.status = rc;
    }
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(own);
    }
    return rc;
}

extern "C" int ghsvd_solve(int m, int n, int p, const double *F, int ldf, const int8_t *J,
                           const double *G, int ldg, double *lambda, double *X, int ldx,
                           void *work, size_t lwork, const ghsvd_options *opt, ghsvd_info *info,
                           void *stream) {
    ghsvd_options o;
    fill_options(opt, o);
    if (!valid_sizes(m, n, p) || ldf < m || ldg < p || ldx < n || !F || !J || !G || !lambda ||
        !X || !valid_options(o)) {
        if (info) {
            *info = ghsvd_info{};
            info->status = GHSVD_EINVAL;
        }
        return GHSVD_EINVAL;
    }
    std::vector<PencilIO> io(1);
    io[0] = PencilIO{m, n, p, reinterpret_cast<const double2 *>(F), ldf, J,
                     reinterpret_cast<const double2 *>(G), ldg, lambda,
                     reinterpret_cast<double2 *>(X), ldx};
    std::vector<ghsvd_info> inf;
    const int rc = run_with_workspace(io, o, work, lwork, inf, reinterpret_cast<hipStream_t>(stream));
    if (info) {
        *info = inf.empty() ? ghsvd_info{} : inf[0];
        if (inf.empty()) info->status = rc;
    }
    return rc;
}

extern "C" int ghsvd_solve_batched(int batch, const int *m, const int *n, const int *p,
                                   const double *const *F, const int *ldf, const int8_t *const *J,
                                   const double *const *G, const int *ldg, double *const *lambda,
                                   double *const *X, const int *ldx, void *work, size_t lwork,
                                   const ghsvd_options *opt, ghsvd_info *info, void *stream) {
    if (batch < 1 || !m || !n || !p || !F || !ldf || !J || !G || !ldg || !lambda || !X || !ldx)
        return GHSVD_EINVAL;
    ghsvd_options o;
    fill_options(opt, o);
    if (!valid_options(o)) return GHSVD_EINVAL;
    // The workspace is sized by ghsvd_workspace_size_batched over all pencils;
    // a pencil with invalid arguments gets GHSVD_EINVAL and no work.
    std::vector<PencilIO> io;
    std::vector<int> map;
    std::vector<int> st(batch, GHSVD_OK);
    for (int k = 0; k < batch; ++k) {
        if (!valid_sizes(m[k], n[k], p[k]) || ldf[k] < m[k] || ldg[k] < p[k] || ldx[k] < n[k] ||
            !F[k] || !J[k] || !G[k] || !lambda[k] || !X[k]) {
            st[k] = GHSVD_EINVAL;
            continue;
        }
        io.push_back(PencilIO{m[k], n[k], p[k], reinterpret_cast<const double2 *>(F[k]), ldf[k], J[k],
                              reinterpret_cast<const double2 *>(G[k]), ldg[k], lambda[k],
                              reinterpret_cast<double2 *>(X[k]), ldx[k]});
        map.push_back(k);
    }
    std::vector<ghsvd_info> inf;
    int rc = GHSVD_OK;
    if (!io.empty())
        rc = run_with_workspace(io, o, work, lwork, inf, reinterpret_cast<hipStream_t>(stream));
    int worst = (rc == GHSVD_EDEVICE || rc == GHSVD_ENOMEM) ? rc : GHSVD_OK;
    if (info)
        for (int k = 0; k < batch; ++k) {
            info[k] = ghsvd_info{};
            info[k].status = st[k];
        }
    for (size_t q = 0; q < map.size(); ++q) {
        if (q < inf.size()) st[map[q]] = inf[q].status;
        if (info && q < inf.size()) info[map[q]] = inf[q];
    }
    for (int k = 0; k < batch; ++k) worst = worst_of(worst, st[k]);
    return worst;
}

extern "C" int ghsvd_reduce(int m, int n, int p, const double *F, int ldf, const int8_t *J,
                            const double *G, int ldg, double *Fsq, int ldfs, int8_t *Jsq,
                            double *Gsq, int ldgs, int *perm, int *n2x2, void *stream) {
    if (!valid_sizes(m, n, p) || ldf < m || ldg < p || ldfs < n || ldgs < n || !F || !J || !G ||
        !Fsq || !Jsq || !Gsq || !perm)
        return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ghsvd_options o;
    fill_options(nullptr, o);
    Plan pl = make_plan(m, n, p, o, 8);
    pl.reduce = 1;
    pl.mr = n;
    pl.pr = n;
    pl.ldf = pad_ld(n);
    pl.ldg = pad_ld(n);
    OwnedBatch ob;
    const size_t need = batch_bytes(1) + pencil_bytes(pl);
    GHSVD_HIP(hipMalloc(&ob.buf, need));
    Carver c{reinterpret_cast<char *>(ob.buf), 0, need};
    carve_batch(c, ob.bc, 1);
    ob.bc.B = 1;
    ob.bc.host.resize(1);
    PencilDev &d = ob.bc.host[0];
    d = PencilDev{};
    c.used = align_up(c.used, 256);
    carve_pencil(c, pl, d);
    d.Fin = reinterpret_cast<const double2 *>(F);
    d.ldfin = ldf;
    d.Jin = J;
    d.Gin = reinterpret_cast<const double2 *>(G);
    d.ldgin = ldg;
    int rc = upload_batch(ob.bc, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, s, ob.bc.dev, 1);
    if ((rc = check_inputs(m, n, p, d.Fin, ldf, J, d.Gin, ldg, d.small, d.gnorm2, s))) return rc;
    std::vector<int> fl;
    if ((rc = gather_small(ob.bc, 0, fl, s))) return rc;
    if (fl[0] & 1) return GHSVD_EINVAL;
    if (fl[0] & 2) return GHSVD_ENONFINITE;
    std::vector<int> rst, n2;
    if ((rc = run_reduction(ob.bc, rst, n2, s))) return rc;
    if (n2x2) *n2x2 = n2[0];
    if (rst[0]) return rst[0];
    if ((rc = jqr_extract(d, reinterpret_cast<double2 *>(Fsq), ldfs, nullptr, s))) return rc;
    if ((rc = copy_cols(n, n, d.Gt, d.ldgt, reinterpret_cast<double2 *>(Gsq), ldgs, d.perm, s)))
        return rc;
    GHSVD_HIP(hipMemcpyAsync(Jsq, d.Jw, (size_t)n, hipMemcpyDeviceToDevice, s));
    GHSVD_HIP(hipMemcpyAsync(perm, d.perm, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    return GHSVD_OK;
}

extern "C" int ghsvd_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G,
                            int ldg, double *Z, int ldz, int nsweeps, int waves_per_pair,
                            int crit_literal, long long *counters, int *sweeps_done,
                            void *stream) {
    if (n < 1 || m < 1 || p < 1 || ldf < m || ldg < p || ldz < n || nsweeps < 1 ||
        nsweeps > kMaxHist || n_plus < 0 || n_plus > m || !F || !G || !Z || waves_per_pair < 0 ||
        waves_per_pair > 16)
        return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    OwnedBatch ob;
    int rc = make_inplace_batch(ob, m, n, p, F, ldf, G, ldg, Z, ldz, 0, 8, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_set_nplus, dim3(1), dim3(1), 0, s, ob.bc.dev, n_plus);
    std::vector<SweepResult> res;
    rc = run_pointwise_stage(ob.bc, 0, nsweeps, crit_literal,
                             choose_pair_geom(m > p ? m : p, waves_per_pair), s, res);
    if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) return rc;
    if ((rc = copy_counters(ob.bc, nsweeps, counters, sweeps_done, s))) return rc;
    return res[0].status;
}

static int block_sweeps_args_ok(int m, int n, int p, const double *F, int ldf, int n_plus,
                                const double *G, int ldg, const double *Z, int ldz,
                                int block_width, int inner_order, int nsweeps) {
    if (n < 4 || m < 1 || p < 1 || ldf < m || ldg < p || ldz < n || nsweeps < 1 ||
        nsweeps > kMaxHist || n_plus < 0 || n_plus > m || !F || !G || !Z)
        return 0;
    if (block_width != 0 && block_width != 8 && block_width != 16 && block_width != 32) return 0;
    return inner_order == GHSVD_INNER_FULL || inner_order == GHSVD_INNER_CROSS ||
           inner_order == GHSVD_INNER_FB || inner_shortened(inner_order);
}

// The blocked stage on a prepared one-pencil in-place batch.
static int block_sweeps_on(const BatchCtx &bc, int n_plus, int inner_order, int nsweeps,
                           int crit_literal, long long *counters, int *sweeps_done,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_set_nplus, dim3(1), dim3(1), 0, s, bc.dev, n_plus);
    GHSVD_HIP(hipGetLastError());
    std::vector<SweepResult> res;
    int rc = run_blocked_stage(bc, 0, nsweeps, crit_literal, inner_order, s, res);
    if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) return rc;
    if ((rc = copy_counters(bc, nsweeps, counters, sweeps_done, s))) return rc;
    return res[0].status;
}

extern "C" int ghsvd_block_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G,
                                  int ldg, double *Z, int ldz, int block_width, int inner_order,
                                  int nsweeps, int crit_literal, long long *counters,
                                  int *sweeps_done, void *stream) {
    if (!block_sweeps_args_ok(m, n, p, F, ldf, n_plus, G, ldg, Z, ldz, block_width, inner_order,
                              nsweeps))
        return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    OwnedBatch ob;
    int rc = make_inplace_batch(ob, m, n, p, F, ldf, G, ldg, Z, ldz, 1,
                                pick_block_width(n, block_width), s, inner_shortened(inner_order));
    if (rc) return rc;
    return block_sweeps_on(ob.bc, n_plus, inner_order, nsweeps, crit_literal, counters,
                           sweeps_done, s);
}

// ---------------------------------------------------------------------------
// Allocation-free blocked sweeps.  All scratch of ghsvd_block_sweeps_noalloc
// (descriptor, prefix sums, done flags, sweep state, counters, partial Grams,
// block transforms) is carved from this library-owned device array: one copy
// per GPU, held until the process ends.  In host code the array's name is a
// host-side stand-in, not a device address; the address of the current
// device's copy comes from hipGetSymbolAddress, once per device, and only
// that address is passed to kernels and copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GHSVD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];  // held for a whole call on that device
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch copy (looked up on the
// first call on each device).  The caller holds g_scratch_mu[dev].
static int scratch_address(int dev, void **ptr) {
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a)
            return GHSVD_EDEVICE;
        g_scratch_ptr[dev] = a;
    }
    *ptr = g_scratch_ptr[dev];
    return GHSVD_OK;
}

extern "C" int ghsvd_block_sweeps_noalloc(int m, int n, int p, double *F, int ldf, int n_plus,
                                          double *G, int ldg, double *Z, int ldz, int block_width,
                                          int inner_order, int nsweeps, int crit_literal,
                                          long long *counters, int *sweeps_done, void *stream) {
    if (!block_sweeps_args_ok(m, n, p, F, ldf, n_plus, G, ldg, Z, ldz, block_width, inner_order,
                              nsweeps) ||
        inner_shortened(inner_order))
        return GHSVD_EINVAL;
    const int w = pick_block_width(n, block_width);
    if (inplace_bytes(m, n, p, 1, w) > (size_t)GHSVD_NOALLOC_SCRATCH_BYTES) return GHSVD_ENOMEM;
    int dev = -1;
    GHSVD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return GHSVD_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    void *buf = nullptr;
    int rc = scratch_address(dev, &buf);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    BatchCtx bc;
    bc.plain = true;
    if ((rc = inplace_batch_at(bc, buf, GHSVD_NOALLOC_SCRATCH_BYTES, m, n, p, F, ldf, G, ldg, Z,
                               ldz, 1, w, s)))
        return rc;
    return block_sweeps_on(bc, n_plus, inner_order, nsweeps, crit_literal, counters, sweeps_done,
                           s);
}

extern "C" int ghsvd_autotune(int batch, const int *m, const int *n, const int *p,
                              const double *const *F, const int *ldf, const int8_t *const *J,
                              const double *const *G, const int *ldg, void *work, size_t lwork,
                              const ghsvd_options *opt, int *block_width, int *waves_per_pair,
                              float *trial_ms, void *stream) {
    if (batch < 1 || !m || !n || !p || !F || !ldf || !J || !G || !ldg) return GHSVD_EINVAL;
    ghsvd_options o;
    fill_options(opt, o);
    if (!valid_options(o)) return GHSVD_EINVAL;
    std::vector<PencilIO> io;
    int max_n = 0;
    for (int k = 0; k < batch; ++k) {
        if (!valid_sizes(m[k], n[k], p[k]) || ldf[k] < m[k] || ldg[k] < p[k] || !F[k] || !J[k] ||
            !G[k])
            return GHSVD_EINVAL;
        io.push_back(PencilIO{m[k], n[k], p[k], reinterpret_cast<const double2 *>(F[k]), ldf[k], J[k],
                              reinterpret_cast<const double2 *>(G[k]), ldg[k], nullptr, nullptr,
                              n[k]});
        max_n = std::max(max_n, n[k]);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ghsvd_options ao = o;
    ao.block_width = 0;
    const size_t need = solve_batch_bytes(io, ao);
    void *own = nullptr;
    if (!work) {
        if (hipMalloc(&own, need) != hipSuccess) return GHSVD_EDEVICE;
        work = own;
        lwork = need;
    }
    struct Free {
        void *p;
        hipStream_t s;
        ~Free() {
            if (p) {
                (void)hipStreamSynchronize(s);
                (void)hipFree(p);
            }
        }
    } fr{own, s};
    if (lwork < need) return GHSVD_ENOMEM;
    // one FP64 sweep per candidate on these pencils, timed by stage
    static const int kWpp[4] = {1, 2, 4, 8};
    static const int kW[3] = {8, 16, 32};
    float t[7] = {-1, -1, -1, -1, -1, -1, -1};
    int best_wpp = 0, best_w = pick_block_width(max_n, 0);
    float best = 0.0f;
    for (int i = 0; i < 4; ++i) {
        ghsvd_options to = o;
        to.precision = GHSVD_FP64;
        to.variant = GHSVD_POINTWISE;
        to.waves_per_pair = kWpp[i];
        to.max_sweeps = 1;
        StageClock ck;
        std::vector<ghsvd_info> inf;
        const int rc = solve_batch(io, to, work, lwork, inf, s, &ck);
        if (rc < 0) return rc;
        t[i] = ck.pointwise_ms;
        if (best_wpp == 0 || t[i] < best) {
            best = t[i];
            best_wpp = kWpp[i];
        }
    }
    if (o.variant == GHSVD_BLOCKED) {
        best = 0.0f;
        int bw = 0;
        for (int j = 0; j < 3; ++j) {
            ghsvd_options to = o;
            to.precision = GHSVD_FP64;
            to.block_width = kW[j];
            to.waves_per_pair = best_wpp;
            to.max_sweeps = 1;
            StageClock ck;
            std::vector<ghsvd_info> inf;
            const int rc = solve_batch(io, to, work, lwork, inf, s, &ck);
            if (rc < 0) return rc;
            t[4 + j] = ck.blocked_ms;
            if (bw == 0 || t[4 + j] < best) {
                best = t[4 + j];
                bw = kW[j];
            }
        }
        best_w = bw;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(io, o)] = TuneVal{best_w, best_wpp};
    }
    if (block_width) *block_width = best_w;
    if (waves_per_pair) *waves_per_pair = best_wpp;
    if (trial_ms)
        for (int i = 0; i < 7; ++i) trial_ms[i] = t[i];
    return GHSVD_OK;
}

extern "C" void ghsvd_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}
