// pair_sweep.hip -- the pointwise pivot-pair kernel and its sweep driver.
//
// One workgroup per pivot pair of a round-robin step (Section 6.3: the pairs
// of a step are disjoint, so they run concurrently).  A workgroup reads its
// two columns of F and G once (coalesced: consecutive lanes read consecutive
// rows of a column-major matrix), forms the six entries of (6.1) with the
// split signature J = diag(I, -I) (Section 4.5.1 run-length form with one
// negative block), reduces them over the wavefronts and the workgroup in a
// fixed order, computes the FP64 2x2 step of Section 6.1 (every wavefront
// redundantly, so no broadcast is needed), and applies Z' to the columns
// still held in registers, then to the two columns of Z.
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

template <typename T, int NT, int R>
__global__ __launch_bounds__(NT) void k_pair(SweepArgs A, int step) {
    using C2 = typename Cplx<T>::type;
    if (A.st->done) return;
    const int slot = blockIdx.x;
    int p, q;
    rr_pair(A.N, step, slot, p, q);
    if (q >= A.n) return;  // bye slot of an odd order
    const int tid = threadIdx.x;

    C2 *Fp = reinterpret_cast<C2 *>(A.F) + (size_t)p * A.ldf;
    C2 *Fq = reinterpret_cast<C2 *>(A.F) + (size_t)q * A.ldf;
    C2 *Gp = reinterpret_cast<C2 *>(A.G) + (size_t)p * A.ldg;
    C2 *Gq = reinterpret_cast<C2 *>(A.G) + (size_t)q * A.ldg;
    C2 *Zp_ = reinterpret_cast<C2 *>(A.Z) + (size_t)p * A.ldz;
    C2 *Zq = reinterpret_cast<C2 *>(A.Z) + (size_t)q * A.ldz;

    constexpr int RR = R > 0 ? R : 1;
    C2 fp[RR], fq[RR], gp[RR], gq[RR];
    T a = 0, b = 0, cr = 0, ci = 0, sa = 0, sb = 0, sr = 0, si = 0;
    const int m = A.m, pr = A.p, nplus = A.nplus;
    if constexpr (R > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < m) {
                fp[r] = Fp[i];
                fq[r] = Fq[i];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < pr) {
                gp[r] = Gp[i];
                gq[r] = Gq[i];
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
            acc_pair<T, C2>(Fp[i], Fq[i], i < nplus ? T(1) : T(-1), a, b, cr, ci);
        for (int i = tid; i < pr; i += NT) acc_pair<T, C2>(Gp[i], Gq[i], T(1), sa, sb, sr, si);
    }

    __shared__ double red[8 * (NT / kWave)];
    double v[8] = {(double)a, (double)b, (double)cr, (double)ci,
                   (double)sa, (double)sb, (double)sr, (double)si};
    block_sum<8>(v, red);

    Zp z;
    int kind = hz_step(v[0], v[1], cmk(v[2], v[3]), v[4], v[5], cmk(v[6], v[7]), A.tol, A.crit, z,
                       A.fp32);
    // FP32 stage: a pair that looks dependent in FP32 is left to the FP64 sweeps.
    if (A.fp32 && kind == GHSVD_ERANK) kind = kSkip;
    if (tid == 0) {
        unsigned long long *c = A.slot_cnt + 3 * slot;
        c[0] += 1ull;
        c[1] += (kind > 0) ? 1ull : 0ull;
        c[2] += (kind == kBig) ? 1ull : 0ull;
        if (kind < 0) atomicCAS(&A.st->err, 0, kind);
    }
    if (kind <= 0) return;

    const C2 z11 = cvt<T>(z.z11), z21 = cvt<T>(z.z21), z12 = cvt<T>(z.z12), z22 = cvt<T>(z.z22);
    if constexpr (R > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + r * NT;
            if (i < m) {
                Fp[i] = upd(fp[r], fq[r], z11, z21);
                Fq[i] = upd(fp[r], fq[r], z12, z22);
            }
            if (i < pr) {
                Gp[i] = upd(gp[r], gq[r], z11, z21);
                Gq[i] = upd(gp[r], gq[r], z12, z22);
            }
        }
    } else {
        for (int i = tid; i < m; i += NT) {
            const C2 xp = Fp[i], xq = Fq[i];
            Fp[i] = upd(xp, xq, z11, z21);
            Fq[i] = upd(xp, xq, z12, z22);
        }
        for (int i = tid; i < pr; i += NT) {
            const C2 xp = Gp[i], xq = Gq[i];
            Gp[i] = upd(xp, xq, z11, z21);
            Gq[i] = upd(xp, xq, z12, z22);
        }
    }
    for (int i = tid; i < A.n; i += NT) {
        const C2 xp = Zp_[i], xq = Zq[i];
        Zp_[i] = upd(xp, xq, z11, z21);
        Zq[i] = upd(xp, xq, z12, z22);
    }
}

// End of a sweep: sums the per-slot counters (fixed order), records them,
// clears them, and sets the convergence flag (Section 6.1.7: stop after a
// sweep without big transformations; Algorithm 2: stop at the sweep cap).
__global__ __launch_bounds__(256) void k_end_sweep(SweepState *st, unsigned long long *cnt,
                                                   int nslots) {
    __shared__ double red[3 * 4];
    if (st->done) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        v[0] += (double)cnt[3 * s + 0];
        v[1] += (double)cnt[3 * s + 1];
        v[2] += (double)cnt[3 * s + 2];
        cnt[3 * s + 0] = 0ull;
        cnt[3 * s + 1] = 0ull;
        cnt[3 * s + 2] = 0ull;
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
    }
}

__global__ void k_reset_state(SweepState *st, unsigned long long *cnt, int nslots, int max_sweeps,
                              int noise_floor) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = t; s < 3 * nslots; s += gridDim.x * blockDim.x) cnt[s] = 0ull;
    if (t == 0) {
        st->done = 0;
        st->sweeps = 0;
        st->err = 0;
        st->converged = 0;
        st->max_sweeps = max_sweeps;
        st->noise_floor = noise_floor;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

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

int enqueue_end_sweep(SweepState *st, unsigned long long *cnt, int nslots, hipStream_t stream) {
    hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(256), 0, stream, st, cnt, nslots);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

int enqueue_reset_state(SweepState *st, unsigned long long *slot_cnt, int nslots,
                        int max_sweeps, hipStream_t stream, int noise_floor) {
    int blocks = (3 * nslots + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_reset_state, dim3(blocks), dim3(256), 0, stream, st, slot_cnt, nslots,
                       max_sweeps, noise_floor);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

// Pair-kernel timing for measurement harnesses (see ghsvd_profile_enable).
namespace prof {
static std::mutex mu;
static int every = 0;
static long long launches = 0;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
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

void launch_pair_step(PairFn fn, const SweepArgs &a, PairGeom g, int step, hipStream_t stream) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    {
        std::lock_guard<std::mutex> lk(prof::mu);
        if (prof::every > 0) {
            if (prof::launches % prof::every == 0) {
                e0 = prof::take_event();
                e1 = prof::take_event();
            }
            prof::launches++;
        }
    }
    if (e0 && e1) (void)hipEventRecord(e0, stream);
    hipLaunchKernelGGL(fn, dim3(a.nslots), dim3(g.nt), 0, stream, a, step);
    if (e0 && e1) {
        (void)hipEventRecord(e1, stream);
        std::lock_guard<std::mutex> lk(prof::mu);
        prof::pending.emplace_back(e0, e1);
    }
}

int enqueue_pointwise_sweep(const SweepArgs &a, PairGeom g, hipStream_t stream) {
    PairFn fn = a.fp32 ? pick<float>(g.nt, g.r) : pick<double>(g.nt, g.r);
    if (!fn) return GHSVD_EINVAL;
    const int steps = a.N - 1;
    for (int s = 0; s < steps; ++s) launch_pair_step(fn, a, g, s, stream);
    hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(256), 0, stream, a.st, a.slot_cnt, a.nslots);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

void trace_stage(const char *name, const SweepState &hs) {
    if (!std::getenv("GHSVD_TRACE")) return;
    for (int k = 0; k < hs.sweeps && k < kMaxHist; ++k)
        std::fprintf(stderr, "ghsvd %s sweep %d: visited %llu transformed %llu big %llu\n", name,
                     k + 1, hs.hist[3 * k], hs.hist[3 * k + 1], hs.hist[3 * k + 2]);
}

int run_pointwise_sweeps(SweepArgs a, int max_sweeps, PairGeom g, hipStream_t stream,
                         SweepResult &res) {
    res = SweepResult{GHSVD_OK, 0, 0, 0, 0, 0};
    if (a.n < 2) {
        res.converged = 1;
        return GHSVD_OK;
    }
    int rc = enqueue_reset_state(a.st, a.slot_cnt, a.nslots, max_sweeps, stream, a.fp32);
    if (rc) return rc;
    SweepState hs;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        rc = enqueue_pointwise_sweep(a, g, stream);
        if (rc) return rc;
        GHSVD_HIP(hipMemcpyAsync(&hs, a.st, offsetof(SweepState, hist), hipMemcpyDeviceToHost,
                                 stream));
        GHSVD_HIP(hipStreamSynchronize(stream));
        if (hs.done) break;
    }
    GHSVD_HIP(hipMemcpyAsync(&hs, a.st, sizeof(SweepState), hipMemcpyDeviceToHost, stream));
    GHSVD_HIP(hipStreamSynchronize(stream));
    trace_stage(a.fp32 ? "pointwise-fp32" : "pointwise-fp64", hs);
    res.sweeps = hs.sweeps;
    res.converged = hs.converged;
    for (int s = 0; s < hs.sweeps && s < kMaxHist; ++s) {
        res.visited += (long long)hs.hist[3 * s + 0];
        res.transformed += (long long)hs.hist[3 * s + 1];
        res.big += (long long)hs.hist[3 * s + 2];
    }
    if (hs.err) res.status = hs.err;
    else res.status = hs.converged ? GHSVD_OK : GHSVD_NOT_CONVERGED;
    return res.status;
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

extern "C" int ghsvd_sweeps(int m, int n, int p, double *F, int ldf, int n_plus, double *G,
                            int ldg, double *Z, int ldz, int nsweeps, int waves_per_pair,
                            int crit_literal, long long *counters, int *sweeps_done,
                            void *stream) {
    if (n < 1 || m < 1 || p < 1 || ldf < m || ldg < p || ldz < n || nsweeps < 1 || n_plus < 0 ||
        n_plus > m || !F || !G || !Z)
        return GHSVD_EINVAL;
    if (nsweeps > kMaxHist) return GHSVD_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int N = n + (n & 1);
    SweepState *st = nullptr;
    unsigned long long *cnt = nullptr;
    GHSVD_HIP(hipMalloc(&st, sizeof(SweepState)));
    if (hipMalloc(&cnt, sizeof(unsigned long long) * 3 * (N / 2 + 1)) != hipSuccess) {
        (void)hipFree(st);
        return GHSVD_EDEVICE;
    }
    SweepArgs a{};
    a.F = F; a.ldf = ldf; a.m = m; a.nplus = n_plus;
    a.G = G; a.ldg = ldg; a.p = p;
    a.Z = Z; a.ldz = ldz; a.n = n;
    a.N = N; a.nslots = N / 2;
    a.tol = 0x1p-52 * sqrt((double)n);
    a.crit = crit_literal;
    a.fp32 = 0;
    a.slot_cnt = cnt;
    a.st = st;
    const int rows = m > p ? m : p;
    SweepResult r;
    int rc = run_pointwise_sweeps(a, nsweeps, choose_pair_geom(rows, waves_per_pair), s, r);
    if (rc < 0 && rc != GHSVD_ERANK && rc != GHSVD_ENONFINITE) {
        (void)hipFree(st);
        (void)hipFree(cnt);
        return rc;
    }
    SweepState hs;
    if (hipMemcpy(&hs, st, sizeof(SweepState), hipMemcpyDeviceToHost) == hipSuccess) {
        if (counters)
            for (int k = 0; k < nsweeps; ++k)
                for (int j = 0; j < 3; ++j)
                    counters[3 * k + j] = k < hs.sweeps ? (long long)hs.hist[3 * k + j] : 0;
        if (sweeps_done) *sweeps_done = hs.sweeps;
    }
    (void)hipFree(st);
    (void)hipFree(cnt);
    return r.status;
}

extern "C" void ghsvd_profile_enable(int every) {
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::every = every > 0 ? every : 0;
    prof::launches = 0;
}

extern "C" int ghsvd_profile_read(double *ms, long long *timed, long long *launches) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    long long nl;
    {
        std::lock_guard<std::mutex> lk(prof::mu);
        ev.swap(prof::pending);
        nl = prof::launches;
        prof::launches = 0;
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
