// batched.hip -- many independent pencils of uneven order in one call.
#include <vector>

#include "solver.hpp"

namespace ghsvd {

static void fill_opts(const ghsvd_options *opt, ghsvd_options &o) {
    ghsvd_default_options(&o);
    if (opt) o = *opt;
    if (o.max_sweeps <= 0) o.max_sweeps = kDefaultMaxSweeps;
    if (o.max_sweeps > kMaxHist) o.max_sweeps = kMaxHist;
}

}  // namespace ghsvd

using namespace ghsvd;

extern "C" size_t ghsvd_workspace_size_batched(int batch, const int *m, const int *n, const int *p,
                                               const ghsvd_options *opt) {
    if (batch < 1 || !m || !n || !p) return 0;
    ghsvd_options o;
    fill_opts(opt, o);
    size_t total = 0;
    for (int k = 0; k < batch; ++k) {
        if (n[k] < 1 || m[k] < n[k] || p[k] < n[k]) return 0;
        total += plan_bytes(make_plan(m[k], n[k], p[k], o));
    }
    return total;
}

extern "C" int ghsvd_solve_batched(int batch, const int *m, const int *n, const int *p,
                                   const double *const *F, const int *ldf, const int8_t *const *J,
                                   const double *const *G, const int *ldg, double *const *lambda,
                                   double *const *X, const int *ldx, void *work, size_t lwork,
                                   const ghsvd_options *opt, ghsvd_info *info, void *stream) {
    if (batch < 1 || !m || !n || !p || !F || !ldf || !J || !G || !ldg || !lambda || !X || !ldx)
        return GHSVD_EINVAL;
    ghsvd_options o;
    fill_opts(opt, o);
    const size_t need = ghsvd_workspace_size_batched(batch, m, n, p, &o);
    if (need == 0) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void *own = nullptr;
    if (!work) {
        GHSVD_HIP(hipMalloc(&own, need));
        work = own;
        lwork = need;
    }
    if (lwork < need) return GHSVD_ENOMEM;
    Carver c{reinterpret_cast<char *>(work), 0, lwork};
    int worst = GHSVD_OK;
    for (int k = 0; k < batch; ++k) {
        ghsvd_info inf{};
        int rc;
        if (ldf[k] < m[k] || ldg[k] < p[k] || ldx[k] < n[k] || !F[k] || !J[k] || !G[k] ||
            !lambda[k] || !X[k]) {
            rc = GHSVD_EINVAL;
        } else {
            const Plan pl = make_plan(m[k], n[k], p[k], o);
            Carver ck{c.base + align_up(c.used, 256), 0, lwork - align_up(c.used, 256)};
            PencilWs w = carve(ck, pl);
            c.used = align_up(c.used, 256) + ck.used;
            rc = solve_one(pl, w, reinterpret_cast<const double2 *>(F[k]), ldf[k], J[k],
                           reinterpret_cast<const double2 *>(G[k]), ldg[k], lambda[k],
                           reinterpret_cast<double2 *>(X[k]), ldx[k], o, inf, s);
        }
        inf.status = rc;
        if (info) info[k] = inf;
        if (rc < 0 || worst < 0) worst = (rc < worst) ? rc : worst;
        else if (rc > worst) worst = rc;
    }
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(own);
    }
    return worst;
}
