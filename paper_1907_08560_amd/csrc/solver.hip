// solver.hip -- the C entry points: workspace planning, the reduction, the
// sweep stages and the outputs for one pencil (ghsvd_solve) and for a batch
// of uneven pencils (ghsvd_solve_batched, in batched.hip).
#include <cstdio>
#include <cstring>

#include "post.hpp"
#include "reduce.hpp"
#include "solver.hpp"
#include "sweep.hpp"

namespace ghsvd {

Plan make_plan(int m, int n, int p, const ghsvd_options &o) {
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
    return pl;
}

PencilWs carve(Carver &c, const Plan &pl) {
    PencilWs w{};
    const int n = pl.n;
    if (pl.reduce) {
        w.Ft = c.take<double2>((size_t)pl.ldft * n);
        w.Gt = c.take<double2>((size_t)pl.ldgt * n);
        w.jq.st = c.take<JqrState>(1);
        w.jq.hd = c.take<double>(n);
        w.jq.hc = c.take<double2>(n);
        w.jq.hi = c.take<double>(n);
        w.jq.s = c.take<double2>(2 * (size_t)pl.m);
        w.qv = c.take<double2>(pl.p);
        w.qcoef = c.take<double>(1);
    }
    w.Jw = c.take<int8_t>(pl.m);
    w.rowmap = c.take<int>(pl.m > n ? pl.m : n);
    w.perm = c.take<int>(n);
    w.Fw = c.take<double2>((size_t)pl.ldf * n);
    w.Gw = c.take<double2>((size_t)pl.ldg * n);
    w.Zw = c.take<double2>((size_t)pl.ldz * n);
    w.st = c.take<SweepState>(1);
    w.slot_cnt = c.take<unsigned long long>(3 * (size_t)(pl.N / 2 + 1));
    w.lam_tmp = c.take<double>(n);
    w.scale = c.take<double>(n);
    w.rank = c.take<int>(n);
    w.small = c.take<int>(8);
    w.gnorm2 = c.take<double>(1);
    if (pl.mixed) {
        w.F32 = c.take<float2>((size_t)pl.ldf * n);
        w.G32 = c.take<float2>((size_t)pl.ldg * n);
        w.Z32 = c.take<float2>((size_t)pl.ldz * n);
    }
    if (pl.blocked || pl.mixed) carve_blocked(c, pl, w);
    return w;
}

size_t plan_bytes(const Plan &pl) {
    Carver c{nullptr, 0, (size_t)-1};
    (void)carve(c, pl);
    return align_up(c.used, 256);
}

__global__ void k_zero_small(int *small, double *gnorm2) {
    const int t = threadIdx.x;
    if (t < 8) small[t] = 0;
    if (t == 0) gnorm2[0] = 0.0;
}

static void fill_options(const ghsvd_options *opt, ghsvd_options &o) {
    ghsvd_default_options(&o);
    if (opt) o = *opt;
    if (o.max_sweeps <= 0) o.max_sweeps = kDefaultMaxSweeps;
    if (o.max_sweeps > kMaxHist) o.max_sweeps = kMaxHist;
}

// Reduction (or plain copies) into the sweep buffers; leaves nplus in small[1].
int prepare_pencil(const Plan &pl, const PencilWs &w, const double2 *F, long ldf,
                   const int8_t *J, const double2 *G, long ldg, hipStream_t s, int *n2x2) {
    const int m = pl.m, n = pl.n, p = pl.p;
    int rc;
    *n2x2 = 0;
    if (pl.reduce) {
        if ((rc = copy_cols(m, n, F, ldf, w.Ft, pl.ldft, nullptr, s))) return rc;
        GHSVD_HIP(hipMemcpyAsync(w.Jw, J, (size_t)m, hipMemcpyDeviceToDevice, s));
        rc = run_jqr(m, n, w.Ft, pl.ldft, w.Jw, w.perm, w.jq, s, n2x2);
        if (rc) return rc;
        if ((rc = copy_cols(p, n, G, ldg, w.Gt, pl.ldgt, w.perm, s))) return rc;
        if ((rc = run_qr(p, n, w.Gt, pl.ldgt, w.qv, w.qcoef, s))) return rc;
        if ((rc = jsplit(n, n, w.Ft, pl.ldft, w.Jw, w.Fw, pl.ldf, w.rowmap, w.small + 1, s)))
            return rc;
        if ((rc = copy_cols(n, n, w.Gt, pl.ldgt, w.Gw, pl.ldg, nullptr, s))) return rc;
    } else {
        if ((rc = jsplit(m, n, F, ldf, J, w.Fw, pl.ldf, w.rowmap, w.small + 1, s))) return rc;
        if ((rc = copy_cols(p, n, G, ldg, w.Gw, pl.ldg, nullptr, s))) return rc;
    }
    return set_identity(n, w.Zw, pl.ldz, 0, s);
}

SweepArgs sweep_args(const Plan &pl, const PencilWs &w, int nplus, const ghsvd_options &o,
                     int fp32) {
    SweepArgs a{};
    a.F = fp32 ? (void *)w.F32 : (void *)w.Fw;
    a.ldf = pl.ldf;
    a.m = pl.mr;
    a.nplus = nplus;
    a.G = fp32 ? (void *)w.G32 : (void *)w.Gw;
    a.ldg = pl.ldg;
    a.p = pl.pr;
    a.Z = fp32 ? (void *)w.Z32 : (void *)w.Zw;
    a.ldz = pl.ldz;
    a.n = pl.n;
    a.N = pl.N;
    a.nslots = pl.N / 2;
    a.tol = (fp32 ? 0x1p-23 : 0x1p-52) * sqrt((double)pl.n);
    a.crit = o.crit_literal;
    a.fp32 = fp32;
    a.slot_cnt = w.slot_cnt;
    a.st = w.st;
    return a;
}

static int worst(int a, int b) {
    if (a < 0 || b < 0) return a < b ? a : b;
    return a > b ? a : b;
}

int solve_one(const Plan &pl, const PencilWs &w, const double2 *F, long ldf, const int8_t *J,
              const double2 *G, long ldg, double *lambda, double2 *X, long ldx,
              const ghsvd_options &o, ghsvd_info &info, hipStream_t s) {
    const int n = pl.n;
    int rc;
    hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, s, w.small, w.gnorm2);
    if ((rc = check_inputs(pl.m, n, pl.p, F, ldf, J, G, ldg, w.small, w.gnorm2, s))) return rc;
    int hsmall[8];
    GHSVD_HIP(hipMemcpyAsync(hsmall, w.small, sizeof(hsmall), hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    if (hsmall[0] & 1) return GHSVD_EINVAL;
    if (hsmall[0] & 2) return GHSVD_ENONFINITE;

    rc = prepare_pencil(pl, w, F, ldf, J, G, ldg, s, &info.n2x2);
    if (rc) return rc;
    GHSVD_HIP(hipMemcpyAsync(hsmall, w.small, sizeof(hsmall), hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    const int nplus = hsmall[1];
    info.m_r = pl.mr;
    info.p_r = pl.pr;
    info.n_plus = nplus;

    int status = GHSVD_OK;
    // Stages: (FP32 warm-up, blocked or pointwise, with its FP64 hand-off) or
    // (FP64 blocked), then FP64 pointwise sweeps decide convergence.
    if (pl.mixed) {
        rc = run_fp32_stage(pl, w, nplus, o, info, s);
        if (rc < 0) return rc;
    } else if (pl.blocked) {
        rc = run_blocked_fp64(pl, w, nplus, o, info, s);
        if (rc < 0) return rc;
    }
    {
        SweepArgs a = sweep_args(pl, w, nplus, o, 0);
        const int rows = pl.mr > pl.pr ? pl.mr : pl.pr;
        SweepResult r;
        rc = run_pointwise_sweeps(a, o.max_sweeps, choose_pair_geom(rows, o.waves_per_pair), s, r);
        info.sweeps_fp64 += r.sweeps;
        info.pairs_visited += r.visited;
        info.pairs_transformed += r.transformed;
        info.pairs_big += r.big;
        if (rc < 0) return rc;
        status = worst(status, rc);
    }
    rc = postprocess(pl.mr, nplus, pl.pr, n, w.Fw, pl.ldf, w.Gw, pl.ldg, w.Zw, pl.ldz,
                     pl.reduce ? w.perm : nullptr, w.gnorm2, o.sort, w.lam_tmp, w.scale, w.rank,
                     w.small + 2, lambda, X, ldx, s);
    if (rc) return rc;
    GHSVD_HIP(hipMemcpyAsync(hsmall, w.small, sizeof(hsmall), hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    if (hsmall[2] & 2) return GHSVD_ENONFINITE;
    if (hsmall[2] & 1) return GHSVD_ERANK;
    return status;
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

extern "C" size_t ghsvd_workspace_size(int m, int n, int p, const ghsvd_options *opt) {
    if (!valid_sizes(m, n, p)) return 0;
    ghsvd_options o;
    fill_options(opt, o);
    return plan_bytes(make_plan(m, n, p, o));
}

extern "C" int ghsvd_solve(int m, int n, int p, const double *F, int ldf, const int8_t *J,
                           const double *G, int ldg, double *lambda, double *X, int ldx,
                           void *work, size_t lwork, const ghsvd_options *opt, ghsvd_info *info,
                           void *stream) {
    ghsvd_info inf{};
    auto finish = [&](int rc) {
        inf.status = rc;
        if (info) *info = inf;
        return rc;
    };
    if (!valid_sizes(m, n, p) || ldf < m || ldg < p || ldx < n || !F || !J || !G || !lambda ||
        !X)
        return finish(GHSVD_EINVAL);
    ghsvd_options o;
    fill_options(opt, o);
    if (o.precision != GHSVD_FP64 && o.precision != GHSVD_MIXED) return finish(GHSVD_EINVAL);
    if (o.variant != GHSVD_POINTWISE && o.variant != GHSVD_BLOCKED) return finish(GHSVD_EINVAL);
    const Plan pl = make_plan(m, n, p, o);
    const size_t need = plan_bytes(pl);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void *own = nullptr;
    if (!work) {
        if (hipMalloc(&own, need) != hipSuccess) return finish(GHSVD_EDEVICE);
        work = own;
        lwork = need;
    }
    if (lwork < need) return finish(GHSVD_ENOMEM);
    Carver c{reinterpret_cast<char *>(work), 0, lwork};
    PencilWs w = carve(c, pl);
    int rc = solve_one(pl, w, reinterpret_cast<const double2 *>(F), ldf, J,
                       reinterpret_cast<const double2 *>(G), ldg, lambda,
                       reinterpret_cast<double2 *>(X), ldx, o, inf, s);
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(own);
    }
    return finish(rc);
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
    o.reduce = 1;
    Plan pl = make_plan(m, n, p, o);
    pl.reduce = 1;
    const size_t need = plan_bytes(pl);
    void *buf = nullptr;
    GHSVD_HIP(hipMalloc(&buf, need));
    Carver c{reinterpret_cast<char *>(buf), 0, need};
    PencilWs w = carve(c, pl);
    int rc = GHSVD_OK;
    hipLaunchKernelGGL(k_zero_small, dim3(1), dim3(64), 0, s, w.small, w.gnorm2);
    rc = check_inputs(m, n, p, reinterpret_cast<const double2 *>(F), ldf, J,
                      reinterpret_cast<const double2 *>(G), ldg, w.small, w.gnorm2, s);
    int hsmall[8] = {0};
    if (!rc && hipMemcpyAsync(hsmall, w.small, sizeof(hsmall), hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = GHSVD_EDEVICE;
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = GHSVD_EDEVICE;
    if (!rc && (hsmall[0] & 1)) rc = GHSVD_EINVAL;
    if (!rc && (hsmall[0] & 2)) rc = GHSVD_ENONFINITE;
    int n2 = 0;
    if (!rc) rc = copy_cols(m, n, reinterpret_cast<const double2 *>(F), ldf, w.Ft, pl.ldft, nullptr, s);
    if (!rc && hipMemcpyAsync(w.Jw, J, (size_t)m, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = GHSVD_EDEVICE;
    if (!rc) rc = run_jqr(m, n, w.Ft, pl.ldft, w.Jw, w.perm, w.jq, s, &n2);
    if (!rc) rc = copy_cols(p, n, reinterpret_cast<const double2 *>(G), ldg, w.Gt, pl.ldgt, w.perm, s);
    if (!rc) rc = run_qr(p, n, w.Gt, pl.ldgt, w.qv, w.qcoef, s);
    if (!rc) rc = copy_cols(n, n, w.Ft, pl.ldft, reinterpret_cast<double2 *>(Fsq), ldfs, nullptr, s);
    if (!rc) rc = copy_cols(n, n, w.Gt, pl.ldgt, reinterpret_cast<double2 *>(Gsq), ldgs, nullptr, s);
    if (!rc && hipMemcpyAsync(Jsq, w.Jw, (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = GHSVD_EDEVICE;
    if (!rc && hipMemcpyAsync(perm, w.perm, sizeof(int) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = GHSVD_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = GHSVD_EDEVICE;
    (void)hipFree(buf);
    if (n2x2) *n2x2 = n2;
    return rc;
}
