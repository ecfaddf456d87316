// shorten.hip -- Level-2 blocked FP64 sweeps with (J)QR-shortened block
// pivots (Section 6.4.2).
//
// Instead of forming the block pivot (H^, S^) as Grams of the tall block
// columns, each block pair's c pivot columns are shortened first: the
// hyperbolic QR of F_C under the pencil's signature (with the diagonal and
// Bunch-Kaufman pivoting of Section 5.2.1) gives the square F^ with its
// signature J^ and pivoting P, and the QR of G_C gives G^; with F^'s columns
// put back in the input order (F~ = F^ P^T, G~ = the triangular factor of
// G_C itself), F~^* J^ F~ = F_C^* J F_C and G~^* G~ = G_C^* G_C.  The inner
// level then runs one-sidedly on (F~, J^, G~) with the 2x2 step of Section
// 6.1 -- one round-robin sweep over the c columns (BO), or sweeps until one
// applies no transformation at all, at most 30 (FB) -- accumulating Z^
// (c x c), which the block-column update applies to F_C, G_C and Z_C.
// The paper recommends this form for ill-conditioned block pivots: the
// inner level never squares their conditioning.
//
// Every block pair of a block step is a small pencil of its own (m_r x c,
// p_r x c), and all of them, over all pencils of the batch, go through the
// batched one-time reduction and pointwise sweep of the whole path in one
// sub-batch.  A block step therefore takes about 3 c + c launches instead of
// three; the stage runs its rounds directly (no captured graph).
//
// With three levels (GHSVD_INNER_ML_BO, GHSVD_INNER_ML_FB) the small pencils
// are swept by the Level-2 blocked stage itself, block width kMlWidth, its
// block pivots formed as Grams and swept once each in the full round-robin
// order: the blocking principle applied once more (Section 6.4).
#include <algorithm>
#include <vector>

#include "reduce.hpp"
#include "solver.hpp"
#include "sweep.hpp"

namespace ghsvd {

// Block pair `bpi` of pencil `pk` at the current block step: blocks a and b
// with ca and cb columns.
struct ShortMap {
    int pk, bpi, a, b, ca, cb;
};

// Column j of the pencil's signature as swept (rows 0..n_plus-1 carry +1).
__global__ void k_short_jsig(const PencilDev *PD, int8_t *const *jsig) {
    const PencilDev P = PD[blockIdx.y];
    const int nplus = P.small[1];
    int8_t *J = jsig[blockIdx.y];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < P.mr; r += gridDim.x * blockDim.x)
        J[r] = r < nplus ? int8_t(1) : int8_t(-1);
}

// Copies the pivot columns of every block pair (block a's, then block b's)
// into its small pencil's input buffers.  grid (row chunks, pivot column,
// small pencil).
__global__ void k_short_gather(const PencilDev *PD, const PencilDev *SD, const ShortMap *map) {
    const ShortMap mp = map[blockIdx.z];
    const PencilDev P = PD[mp.pk];
    const PencilDev Q = SD[blockIdx.z];
    const int cc = blockIdx.y;
    if (cc >= mp.ca + mp.cb) return;
    const int col = cc < mp.ca ? mp.a * P.w + cc : mp.b * P.w + (cc - mp.ca);
    const GPtr<double2> fs(P.Fw + (size_t)col * P.ldf), gs(P.Gw + (size_t)col * P.ldg);
    const GPtr<double2> fd(const_cast<double2 *>(Q.Fin) + (size_t)cc * Q.ldfin);
    const GPtr<double2> gd(const_cast<double2 *>(Q.Gin) + (size_t)cc * Q.ldgin);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < P.mr; r += gridDim.x * blockDim.x)
        fd.st(r, fs.ld(r));
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < P.pr; r += gridDim.x * blockDim.x)
        gd.st(r, gs.ld(r));
}

// No block-column update unless a small pencil of this step transformed
// something: every block pair's transformed count starts at zero.
__global__ void k_short_clear(const PencilDev *PD, int B) {
    if ((int)blockIdx.x >= B) return;
    const PencilDev P = PD[blockIdx.x];
    for (int k = threadIdx.x; k < P.nbp; k += blockDim.x) P.ntr[k] = 0;
}

// A small pencil whose shortening failed fails its pencil.
__global__ void k_short_fail(const PencilDev *PD, int pk, int code) {
    if (threadIdx.x == 0) atomicCAS(&PD[pk].st->err, 0, code);
}

// Z^ of each block pair (c x c, pivot-column order) into the block
// transform the update applies (PB x PB, identity on the padding), and the
// inner level's counters into the block pair's (visited, transformed, big).
__global__ void k_short_collect(const PencilDev *PD, const PencilDev *SD, const ShortMap *map,
                                int PB) {
    const ShortMap mp = map[blockIdx.x];
    const PencilDev P = PD[mp.pk];
    const PencilDev Q = SD[blockIdx.x];
    const int c = Q.n;
    const GPtr<double2> Z(P.zh64 + (size_t)mp.bpi * PB * PB);
    for (int idx = threadIdx.x; idx < PB * PB; idx += blockDim.x) {
        const int i = idx % PB, j = idx / PB;
        double2 z = cmk(i == j ? 1.0 : 0.0, 0.0);
        if (i < c && j < c) z = Q.Zw[i + (size_t)j * Q.ldz];
        Z.st(idx, z);
    }
    if (threadIdx.x == 0) {
        const SweepState *st = Q.st;
        unsigned long long v = 0, t = 0, g = 0;
        for (int s = 0; s < st->sweeps && s < kMaxHist; ++s) {
            v += st->hist[3 * s];
            t += st->hist[3 * s + 1];
            g += st->hist[3 * s + 2];
        }
        P.ntr[mp.bpi] = (int)t;
        unsigned long long *cn = P.bcnt + 3 * mp.bpi;
        cn[0] += v;
        cn[1] += t;
        cn[2] += g;
    }
}

// Plan of one block pair's small pencil: F_C (m_r x c) and G_C (p_r x c),
// always reduced (also when square), swept in FP64 pointwise or by the
// Level-2 blocked stage of width kMlWidth (its scratch is always carved).
static Plan short_plan(int mr, int c, int pr) {
    Plan pl{};
    pl.blocked = 1;
    pl.w = kMlWidth;
    pl.m = mr;
    pl.n = c;
    pl.p = pr;
    pl.reduce = 1;
    pl.mr = c;
    pl.pr = c;
    pl.ldft = pad_ld(mr);
    pl.ldgt = pad_ld(pr);
    pl.ldf = pad_ld(c);
    pl.ldg = pad_ld(c);
    pl.ldz = pad_ld(c);
    pl.N = c + (c & 1);
    return pl;
}

static size_t short_pencil_bytes(int mr, int c, int pr) {
    // the small pencil's own carve, plus its staged input columns
    return pencil_bytes(short_plan(mr, c, pr)) + align_up((size_t)pad_ld(mr) * c * 16, 256) +
           align_up((size_t)pad_ld(pr) * c * 16, 256) + 512;
}

size_t short_stage_bytes(const std::vector<Plan> &outer, int w) {
    size_t total = 0;
    int S = 0;
    for (const Plan &P : outer) {
        int nb = (P.n + w - 1) / w;
        nb += nb & 1;
        S += nb / 2;
        total += (size_t)(nb / 2) * short_pencil_bytes(P.mr, 2 * w, P.pr);
        total += align_up((size_t)P.mr, 256);  // the split signature
    }
    total += batch_bytes(S) + align_up(sizeof(ShortMap) * S, 256) +
             align_up(sizeof(int8_t *) * outer.size(), 256) + 1024;
    return total;
}

struct ShortArg {
    BlkFn upd;        // block-column update kernel of the width
    int upd_nt;
    int crit, fb, ml, PB;
    char *buf;        // the stage's region of the workspace
    size_t cap;
    int8_t **jsig;    // host copy of the per-pencil signature pointers
};

static int short_step(const BatchCtx &c, const void *argp, int step, hipStream_t s) {
    const ShortArg *a = static_cast<const ShortArg *>(argp);
    const int B = c.B;
    hipLaunchKernelGGL(k_short_clear, dim3(B), dim3(256), 0, s, c.dev, B);
    GHSVD_HIP(hipGetLastError());
    std::vector<int> done(B, 0);
    GHSVD_HIP(hipMemcpyAsync(done.data(), c.flag_dev, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    GHSVD_HIP(hipStreamSynchronize(s));
    std::vector<ShortMap> maps;
    for (int k = 0; k < B; ++k) {
        const PencilDev &P = c.host[k];
        if (done[k] || step >= P.nb - 1) continue;
        for (int bpi = 0; bpi < P.nbp; ++bpi) {
            int ba, bb;
            rr_pair(P.nb, step, bpi, ba, bb);
            const int ca = std::max(0, std::min(P.w, P.n - ba * P.w));
            const int cb = std::max(0, std::min(P.w, P.n - bb * P.w));
            if (ca + cb >= 2) maps.push_back(ShortMap{k, bpi, ba, bb, ca, cb});
        }
    }
    const int S = (int)maps.size();
    if (S > 0) {
        // the sub-batch of small pencils, carved afresh for this step's widths
        Carver cv{a->buf, 0, a->cap};
        BatchCtx sub;
        carve_batch(cv, sub, S);
        ShortMap *map_dev = cv.take<ShortMap>(S);
        sub.B = S;
        sub.plain = true;
        // a pointwise FB inner level stops on a sweep with no transformation
        // (Section 6.1.7); a nested blocked level re-forms its block pivots
        // every sweep, so it stops like an outer level, on no big one
        sub.stop_all = a->fb && !a->ml;
        sub.host.resize(S);
        for (int i = 0; i < S; ++i) {
            const PencilDev &P = c.host[maps[i].pk];
            const int cc = maps[i].ca + maps[i].cb;
            PencilDev &d = sub.host[i];
            d = PencilDev{};
            cv.used = align_up(cv.used, 256);
            carve_pencil(cv, short_plan(P.mr, cc, P.pr), d);
            double2 *fin = cv.take<double2>((size_t)pad_ld(P.mr) * cc);
            double2 *gin = cv.take<double2>((size_t)pad_ld(P.pr) * cc);
            d.Fin = fin;
            d.ldfin = pad_ld(P.mr);
            d.Gin = gin;
            d.ldgin = pad_ld(P.pr);
            d.Jin = a->jsig[maps[i].pk];
            d.skip_rank = 1;
        }
        if (!cv.ok()) return GHSVD_ENOMEM;
        int rc = upload_batch(sub, s);
        if (rc) return rc;
        GHSVD_HIP(hipMemcpyAsync(map_dev, maps.data(), sizeof(ShortMap) * S, hipMemcpyHostToDevice,
                                 s));
        int rows = 0;
        for (const PencilDev &P : c.host) rows = std::max(rows, std::max(P.mr, P.pr));
        int bx = (rows + 255) / 256;
        if (bx > 8) bx = 8;
        hipLaunchKernelGGL(k_short_gather, dim3(bx, a->PB, S), dim3(256), 0, s, c.dev, sub.dev,
                           map_dev);
        GHSVD_HIP(hipGetLastError());
        // shortening: the batched one-time reduction of the small pencils
        std::vector<int> rst, n2;
        if ((rc = run_reduction(sub, rst, n2, s))) return rc;
        // a small pencil whose shortening failed fails its pencil and sweeps nothing
        std::vector<int> failed(S, 0);
        for (int i = 0; i < S; ++i) {
            const PencilDev &Q = sub.host[i];
            if ((rc = set_identity(Q.n, Q.Zw, Q.ldz, 0, s))) return rc;
            if (rst[i]) {
                failed[i] = 1;
                hipLaunchKernelGGL(k_short_fail, dim3(1), dim3(64), 0, s, c.dev, maps[i].pk,
                                   rst[i]);
                continue;
            }
            if ((rc = jsplit_map(Q.n, Q.Jw, Q.rowmap, Q.small + 1, s))) return rc;
            if ((rc = jqr_extract(Q, Q.Fw, Q.ldf, Q.rowmap, s, 1))) return rc;
            if ((rc = copy_cols(Q.n, Q.n, Q.Gt, Q.ldgt, Q.Gw, Q.ldg, nullptr, s))) return rc;
        }
        // the inner level: pointwise FP64 sweeps of the small pencils, or the
        // Level-2 blocked stage on them (its own inner level one full
        // round-robin sweep per block pivot), one blocked sweep or sweeps
        // until one applies no big transformation
        std::vector<SweepResult> res;
        if (a->ml)
            rc = run_blocked_stage(sub, 0, a->fb ? kShortFbSweeps : 1, a->crit, GHSVD_INNER_FULL,
                                   s, res, &failed);
        else
            rc = run_pointwise_stage(sub, 0, a->fb ? kShortFbSweeps : 1, a->crit,
                                     choose_pair_geom(a->PB, 0), s, res, &failed);
        if (rc < 0 && rc != GHSVD_ENONFINITE) return rc;
        for (int i = 0; i < S; ++i)
            if (res[i].status < 0)
                hipLaunchKernelGGL(k_short_fail, dim3(1), dim3(64), 0, s, c.dev, maps[i].pk,
                                   res[i].status);
        hipLaunchKernelGGL(k_short_collect, dim3(S), dim3(256), 0, s, c.dev, sub.dev, map_dev,
                           a->PB);
        GHSVD_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(a->upd, dim3(c.total(BatchCtx::kUpd)), dim3(a->upd_nt), 0, s, c.dev,
                       c.pre_of(BatchCtx::kUpd), c.flag_dev, B, step);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

int run_blocked_shortened(const BatchCtx &c, int max_sweeps, int crit, int fb, int ml,
                          hipStream_t s, std::vector<SweepResult> &res) {
    int w = 0, steps = 1;
    for (const PencilDev &P : c.host) {
        if (w == 0) w = P.w;
        if (P.w != w) return GHSVD_EINVAL;
        if (P.nb - 1 > steps) steps = P.nb - 1;
    }
    if (c.total(BatchCtx::kBp) == 0) {
        res.assign(c.B, SweepResult{GHSVD_OK, 0, 1, 0, 0, 0});
        return GHSVD_OK;
    }
    if (!c.short_buf) return GHSVD_ENOMEM;
    // the stage's region: per-pencil signatures first, the rest per step
    Carver cv{c.short_buf, 0, c.short_cap};
    std::vector<int8_t *> jsig(c.B);
    for (int k = 0; k < c.B; ++k) jsig[k] = cv.take<int8_t>((size_t)c.host[k].mr);
    int8_t **jsig_dev = cv.take<int8_t *>(c.B);
    if (!cv.ok()) return GHSVD_ENOMEM;
    GHSVD_HIP(hipMemcpyAsync(jsig_dev, jsig.data(), sizeof(int8_t *) * c.B, hipMemcpyHostToDevice,
                             s));
    int rows = 0;
    for (const PencilDev &P : c.host) rows = std::max(rows, P.mr);
    int bx = (rows + 255) / 256;
    if (bx > 8) bx = 8;
    hipLaunchKernelGGL(k_short_jsig, dim3(bx, c.B), dim3(256), 0, s, c.dev, jsig_dev);
    GHSVD_HIP(hipGetLastError());
    ShortArg a{};
    a.upd = block_update_kernel(w);
    a.upd_nt = 256;
    a.crit = crit;
    a.fb = fb;
    a.ml = ml;
    a.PB = 2 * w;
    cv.used = align_up(cv.used, 256);
    a.buf = c.short_buf + cv.used;
    a.cap = c.short_cap - cv.used;
    a.jsig = jsig.data();
    if (!a.upd) return GHSVD_EINVAL;
    BatchCtx cc = c;
    cc.plain = true;  // host work between the launches of a block step
    return drive_stage(cc, max_sweeps, 0, 1, short_step, &a, steps, "blocked-jqr-fp64", s, res);
}

}  // namespace ghsvd
