// phase1.hip -- Phase 1 (Section 4): the simultaneous factorizations of the
// atom blocks T_a (ZHEBPJ, Sections 4.2-4.3) and the assembly of F~, J~, G~
// (Section 4.4, eq. (4.1)-(4.2)) for gfx950.
//
// ZHEBPJ runs one workgroup per atom: the Hermitian T_a is copied to a
// working matrix of which only the upper triangle is kept, and every pivot
// step (Bunch-Parlett complete pivoting) performs its symmetric interchanges
// on that triangle, forms the pivot's rows of the factor and subtracts the
// rank-1 or rank-2 update from the trailing triangle, finding the next
// step's largest diagonal and off-diagonal moduli in the same pass.  The
// transformation of the pivot block into signs (a block of order 1 scaled by
// |d|^{1/2}, one of order 2 diagonalized by a Jacobi rotation and scaled) is
// folded into the step: with W = diag(|l|^{1/2}) R^* the pivot's rows of the
// factor are [W, J^ Y], Y = diag(|l|^{-1/2}) R^* B, and the Schur complement
// is A22 - Y^* J^ Y, so D^{-1} is never formed.  Factor rows are written by
// original column index, so no interchange touches them, and are reordered
// at the end with the positive signs first (Section 4.3).
//
// The assembly F~_a = M~_a H_a is a batched complex product on FP64 MFMA
// (64 x 64 output tiles, the inner dimension 2 N_L staged through LDS); the
// same workgroups write G~_a = [A_a; U_a B_a] for their tiles.
#include "hz_common.hpp"

#include <climits>
#include <cmath>

namespace ghsvd {
namespace {

constexpr int kBpjThreads = 512;
constexpr int kBpjWaves = kBpjThreads / kWave;
constexpr int kBpjMaxR = 512;

// squared modulus, rounded the same way wherever it is taken (no contraction)
__device__ __forceinline__ double mod2(double2 z) { return __dadd_rn(__dmul_rn(z.x, z.x), __dmul_rn(z.y, z.y)); }

// (value, key) maximum: larger value wins, smaller key among equal values
__device__ __forceinline__ void better(double &v, int &key, double ov, int okey) {
    if (ov > v || (ov == v && okey < key)) { v = ov; key = okey; }
}

// upper-triangle position e of an order-rr triangle (column-major, diagonal
// included) -> (i, j), i <= j
__device__ __forceinline__ void tri_ij(int e, int &i, int &j) {
    int jj = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((jj + 1) * (jj + 2) / 2 <= e) ++jj;
    while (jj * (jj + 1) / 2 > e) --jj;
    j = jj;
    i = e - jj * (jj + 1) / 2;
}

// Two (value, key) maxima over the workgroup; every thread gets both.
__device__ __forceinline__ void block_max2(double &v0, int &k0, double &v1, int &k1, double *lv,
                                           int *lk) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        better(v0, k0, __shfl_xor(v0, off, kWave), __shfl_xor(k0, off, kWave));
        better(v1, k1, __shfl_xor(v1, off, kWave), __shfl_xor(k1, off, kWave));
    }
    if (lane == 0) {
        lv[wid] = v0; lk[wid] = k0;
        lv[kBpjWaves + wid] = v1; lk[kBpjWaves + wid] = k1;
    }
    __syncthreads();
    v0 = lv[0]; k0 = lk[0]; v1 = lv[kBpjWaves]; k1 = lk[kBpjWaves];
    for (int w = 1; w < kBpjWaves; ++w) {
        better(v0, k0, lv[w], lk[w]);
        better(v1, k1, lv[kBpjWaves + w], lk[kBpjWaves + w]);
    }
    __syncthreads();
}

// Symmetric interchange of positions p < q (both >= k) of the Hermitian
// matrix whose upper triangle A holds (rows and columns < k are finished and
// not touched).
__device__ void sym_swap(double2 *A, int r, int k, int p, int q) {
    auto at = [&](int i, int j) -> double2 & { return A[(size_t)j * r + i]; };
    for (int t = threadIdx.x; t < r; t += blockDim.x) {
        if (t >= k && t < p) {  // column entries above p
            const double2 x = at(t, p);
            at(t, p) = at(t, q);
            at(t, q) = x;
        } else if (t > p && t < q) {  // row p against column q, conjugated
            const double2 x = at(p, t);
            at(p, t) = cconj(at(t, q));
            at(t, q) = cconj(x);
        } else if (t > q) {  // rows p and q right of q
            const double2 x = at(p, t);
            at(p, t) = at(q, t);
            at(q, t) = x;
        } else if (t == p) {
            const double2 x = at(p, p);
            at(p, p) = at(q, q);
            at(q, q) = x;
            at(p, q) = cconj(at(p, q));
        }
    }
}

// One atom per workgroup.  T: r x r x atoms (read: upper triangle, real part
// of the diagonal).  Aw, Mw: r x r x atoms working matrices.  Outputs: Mt
// (rows sorted by sign), Jt, piv, stats (2 ints per atom).
__global__ __launch_bounds__(kBpjThreads) void k_p1_bpj(int r, const double2 *T, double2 *Aw,
                                                        double2 *Mw, double2 *Mt,
                                                        signed char *Jt, int *piv, int *stats) {
    __shared__ int perm[kBpjMaxR];
    __shared__ int dest[kBpjMaxR];
    __shared__ signed char sgn[kBpjMaxR];
    __shared__ double2 Y[2][kBpjMaxR];
    __shared__ double lv[2 * kBpjWaves];
    __shared__ int lk[2 * kBpjWaves];
    __shared__ int bad;
    const int a = blockIdx.x, tid = threadIdx.x;
    const size_t rr = (size_t)r * r;
    const double2 *Ta = T + rr * a;
    double2 *A = Aw + rr * a;
    double2 *M = Mw + rr * a;
    if (tid == 0) bad = 0;
    for (int t = tid; t < r; t += blockDim.x) {
        perm[t] = t;
        sgn[t] = 0;
    }
    __syncthreads();
    // copy the upper triangle, clear the factor rows, find the first pivot
    double dv = -1.0, ov = -1.0;
    int dk = INT_MAX, ok = INT_MAX;
    int nonfinite = 0;
    for (size_t e = tid; e < rr; e += blockDim.x) {
        const int i = (int)(e % r), j = (int)(e / r);
        M[e] = cmk(0.0, 0.0);
        if (i > j) continue;
        double2 x = Ta[e];
        if (!isfinite(x.x) || !isfinite(x.y)) nonfinite = 1;
        if (i == j) {
            x.y = 0.0;
            better(dv, dk, __dmul_rn(x.x, x.x), i);
        } else {
            better(ov, ok, mod2(x), j * r + i);
        }
        A[e] = x;
    }
    if (nonfinite) bad = 1;
    block_max2(dv, dk, ov, ok, lv, lk);
    if (bad) {
        for (int t = tid; t < r; t += blockDim.x) {
            Jt[(size_t)a * r + t] = 0;
            piv[(size_t)a * r + t] = t;
        }
        for (size_t e = tid; e < rr; e += blockDim.x) Mt[rr * a + e] = cmk(0.0, 0.0);
        if (tid == 0) {
            stats[2 * a] = GHSVD_ENONFINITE;
            stats[2 * a + 1] = r;
        }
        return;
    }
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    const double a2 = alpha * alpha;
    auto at = [&](int i, int j) -> double2 & { return A[(size_t)j * r + i]; };
    int n2 = 0, k = 0;
    while (k < r) {
        const double mu1 = dv, mu0 = ov > dv ? ov : dv;
        if (!(mu0 > 0.0)) break;  // the Schur complement is zero: signs 0 from k on
        int s, p0, p1 = 0;
        if (mu1 >= a2 * mu0) {
            s = 1;
            p0 = dk;
        } else {
            s = 2;
            p0 = ok % r;
            p1 = ok / r;
        }
        // interchanges: p0 to position k, then p1 to k + 1 (p0 < p1)
        if (p0 != k) sym_swap(A, r, k, k, p0);
        if (tid == 0 && p0 != k) {
            const int x = perm[k];
            perm[k] = perm[p0];
            perm[p0] = x;
        }
        __syncthreads();
        if (s == 2) {
            if (p1 != k + 1) sym_swap(A, r, k, k + 1, p1);
            if (tid == 0 && p1 != k + 1) {
                const int x = perm[k + 1];
                perm[k + 1] = perm[p1];
                perm[p1] = x;
            }
            __syncthreads();
        }
        // the pivot's rows of the factor and Y
        double2 *Mk = M + k, *Mk1 = M + k + 1;
        if (s == 1) {
            const double d = at(k, k).x;
            const double jh = d > 0.0 ? 1.0 : -1.0, sq = sqrt(fabs(d));
            for (int j = k + 1 + tid; j < r; j += blockDim.x) {
                const double2 y = cscale(at(k, j), 1.0 / sq);
                Y[0][j] = y;
                Mk[(size_t)perm[j] * r] = cscale(y, jh);
            }
            if (tid == 0) {
                Mk[(size_t)perm[k] * r] = cmk(sq, 0.0);
                sgn[k] = d > 0.0 ? 1 : -1;
                piv[(size_t)a * r + k] = perm[k];
            }
        } else {
            const double ea = at(k, k).x, eb = at(k + 1, k + 1).x;
            const double2 c = at(k, k + 1);
            const double ac = sqrt(mod2(c));
            const double tau = (eb - ea) / (2.0 * ac);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
            const double2 e = cscale(c, 1.0 / ac);
            const double l1 = ea - t * ac, l2 = eb + t * ac;
            const double j1 = l1 > 0.0 ? 1.0 : -1.0, j2 = l2 > 0.0 ? 1.0 : -1.0;
            const double q1 = sqrt(fabs(l1)), q2 = sqrt(fabs(l2));
            // R^* = [[cs, -sn e], [sn, cs e]]
            for (int j = k + 2 + tid; j < r; j += blockDim.x) {
                const double2 b1 = at(k, j), b2 = cmul(e, at(k + 1, j));
                const double2 y1 = cscale(csub(cscale(b1, cs), cscale(b2, sn)), 1.0 / q1);
                const double2 y2 = cscale(cadd(cscale(b1, sn), cscale(b2, cs)), 1.0 / q2);
                Y[0][j] = y1;
                Y[1][j] = y2;
                Mk[(size_t)perm[j] * r] = cscale(y1, j1);
                Mk1[(size_t)perm[j] * r] = cscale(y2, j2);
            }
            if (tid == 0) {
                Mk[(size_t)perm[k] * r] = cmk(q1 * cs, 0.0);
                Mk[(size_t)perm[k + 1] * r] = cscale(e, -q1 * sn);
                Mk1[(size_t)perm[k] * r] = cmk(q2 * sn, 0.0);
                Mk1[(size_t)perm[k + 1] * r] = cscale(e, q2 * cs);
                sgn[k] = l1 > 0.0 ? 1 : -1;
                sgn[k + 1] = l2 > 0.0 ? 1 : -1;
                piv[(size_t)a * r + k] = -(perm[k] + 1);
                piv[(size_t)a * r + k + 1] = -(perm[k + 1] + 1);
            }
            ++n2;
        }
        __syncthreads();
        // A22 -= Y^* J^ Y on the trailing triangle; next pivot candidates
        const int k2 = k + s, rt = r - k2;
        const double js0 = sgn[k], js1 = s == 2 ? (double)sgn[k + 1] : 0.0;
        dv = -1.0; ov = -1.0; dk = INT_MAX; ok = INT_MAX;
        const int ntri = rt * (rt + 1) / 2;
        for (int e = tid; e < ntri; e += blockDim.x) {
            int ii, jj;
            tri_ij(e, ii, jj);
            const int i = k2 + ii, j = k2 + jj;
            double2 x = at(i, j);
            const double2 yi = Y[0][i], yj = Y[0][j];
            if (i == j) {
                double u = js0 * mod2(yi);
                if (s == 2) u += js1 * mod2(Y[1][i]);
                x = cmk(x.x - u, 0.0);
                better(dv, dk, __dmul_rn(x.x, x.x), i);
            } else {
                double2 u = cscale(cmulc(yi, yj), js0);
                if (s == 2) u = cadd(u, cscale(cmulc(Y[1][i], Y[1][j]), js1));
                x = csub(x, u);
                better(ov, ok, mod2(x), j * r + i);
            }
            at(i, j) = x;
        }
        block_max2(dv, dk, ov, ok, lv, lk);
        k = k2;
    }
    // zero tail: positions k.. keep sign 0 and zero rows
    for (int t = k + tid; t < r; t += blockDim.x) piv[(size_t)a * r + t] = perm[t];
    __syncthreads();
    // inner permutation: positive signs first, then negative, then zero
    if (tid == 0) {
        int np = 0, nn = 0;
        for (int t = 0; t < r; ++t) {
            np += sgn[t] > 0;
            nn += sgn[t] < 0;
        }
        int cp = 0, cn = np, cz = np + nn;
        for (int t = 0; t < r; ++t) dest[t] = sgn[t] > 0 ? cp++ : (sgn[t] < 0 ? cn++ : cz++);
        stats[2 * a] = n2;
        stats[2 * a + 1] = r - np - nn;
    }
    __syncthreads();
    for (int t = tid; t < r; t += blockDim.x) Jt[(size_t)a * r + dest[t]] = sgn[t];
    double2 *Ma = Mt + rr * a;
    for (size_t e = tid; e < rr; e += blockDim.x) {
        const int i = (int)(e % r), j = (int)(e / r);
        Ma[(size_t)j * r + dest[i]] = M[e];
    }
}

// F~_a = M~_a H_a and G~_a = [A_a; U_a B_a], one 64 x 64 output tile per
// workgroup (four wavefronts, one 32 x 32 quarter each, FP64 MFMA 16x16x4:
// A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k; result q of lane l
// at row l / 16 + 4 q, column l % 16 of its 16 x 16 tile).
constexpr int kApTile = 64, kApK = 16;
constexpr int kApStage = kApTile * (kApK + 1) + kApK * (kApTile + 1);  // As and Bs
constexpr int kApOut = kApTile * (kApTile / 2 + 1);                    // half the output tile
constexpr int kApLds = kApStage > kApOut ? kApStage : kApOut;
typedef double p1v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_p1_apply(int r, int nl, int n, const double2 *Mt,
                                                  const double2 *H, int ldh, const double *U,
                                                  double2 *F, int ldf, double2 *G, int ldg) {
    __shared__ double2 lds[kApLds];  // staging, then half the output tile
    double2(*As)[kApK + 1] = reinterpret_cast<double2(*)[kApK + 1]>(lds);
    double2(*Bs)[kApTile + 1] = reinterpret_cast<double2(*)[kApTile + 1]>(lds + kApTile * (kApK + 1));
    double2(*Os)[kApTile / 2 + 1] = reinterpret_cast<double2(*)[kApTile / 2 + 1]>(lds);
    const int a = blockIdx.y, tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
    const int wi = wv & 1, wj = wv >> 1;
    const int nrt = (r + kApTile - 1) / kApTile;
    const int it = blockIdx.x % nrt, jt = blockIdx.x / nrt;
    const int i0 = it * kApTile, c0 = jt * kApTile;
    const double2 *Ma = Mt + (size_t)r * r * a;
    const size_t hrow = (size_t)a * r;
    p1v4d re[2][2], im[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            re[x][y] = p1v4d{0, 0, 0, 0};
            im[x][y] = p1v4d{0, 0, 0, 0};
        }
    const int i16 = lane & 15, kq = lane >> 4;
    for (int k0 = 0; k0 < r; k0 += kApK) {
        for (int e = tid; e < kApTile * kApK; e += blockDim.x) {
            const int row = e % kApTile, kk = e / kApTile;
            const int gi = i0 + row, gk = k0 + kk;
            As[row][kk] = (gi < r && gk < r) ? Ma[(size_t)gk * r + gi] : cmk(0.0, 0.0);
        }
        for (int e = tid; e < kApTile * kApK; e += blockDim.x) {
            const int kk = e % kApK, col = e / kApK;
            const int gk = k0 + kk, gc = c0 + col;
            Bs[kk][col] = (gk < r && gc < n) ? H[(size_t)gc * ldh + hrow + gk] : cmk(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kApK; ks += 4) {
            double2 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = As[wi * 32 + t * 16 + i16][ks + kq];
                bv[t] = Bs[ks + kq][wj * 32 + t * 16 + i16];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].x, bv[y].x, re[x][y], 0, 0, 0);
                    re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[x].y, bv[y].y, re[x][y], 0, 0, 0);
                    im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].x, bv[y].y, im[x][y], 0, 0, 0);
                    im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x].y, bv[y].x, im[x][y], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // store F~ by column halves through LDS (contiguous column segments)
    for (int h = 0; h < 2; ++h) {
        if (wj == h) {
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        Os[wi * 32 + x * 16 + kq + 4 * q][y * 16 + i16] = cmk(re[x][y][q], im[x][y][q]);
        }
        __syncthreads();
        for (int e = tid; e < kApTile * (kApTile / 2); e += blockDim.x) {
            const int row = e % kApTile, col = e / kApTile;
            const int gi = i0 + row, gc = c0 + h * (kApTile / 2) + col;
            if (gi < r && gc < n) F[(size_t)gc * ldf + hrow + gi] = Os[row][col];
        }
        __syncthreads();
    }
    // G~ rows of this tile: A_a copied, B_a scaled by the diagonal of U_a
    for (int e = tid; e < kApTile * kApTile; e += blockDim.x) {
        const int row = e % kApTile, col = e / kApTile;
        const int gi = i0 + row, gc = c0 + col;
        if (gi >= r || gc >= n) continue;
        const double2 x = H[(size_t)gc * ldh + hrow + gi];
        G[(size_t)gc * ldg + hrow + gi] = gi < nl ? x : cscale(x, U[(size_t)a * nl + gi - nl]);
    }
}

size_t bpj_bytes(int atoms, int r) {
    return 2 * align_up((size_t)atoms * r * r * sizeof(double2), 256);
}

int run_bpj(int atoms, int r, const double *T, double *Mt, signed char *Jt, int *piv, int *stats,
            char *work, hipStream_t st) {
    Carver c{work, 0, bpj_bytes(atoms, r)};
    double2 *Aw = c.take<double2>((size_t)atoms * r * r);
    double2 *Mw = c.take<double2>((size_t)atoms * r * r);
    hipLaunchKernelGGL(k_p1_bpj, dim3(atoms), dim3(kBpjThreads), 0, st, r,
                       reinterpret_cast<const double2 *>(T), Aw, Mw, reinterpret_cast<double2 *>(Mt),
                       Jt, piv, stats);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace
}  // namespace ghsvd

using namespace ghsvd;

extern "C" size_t ghsvd_hebpj_workspace_size(int n_atoms, int r) {
    if (n_atoms < 1 || r < 1 || r > kBpjMaxR) return 0;
    return bpj_bytes(n_atoms, r);
}

extern "C" int ghsvd_hebpj_batched(int n_atoms, int r, const double *T, double *Mt,
                                   signed char *Jt, int *piv, int *stats, void *work,
                                   size_t lwork, void *stream) {
    if (n_atoms < 1 || r < 1 || r > kBpjMaxR || !T || !Mt || !Jt || !piv || !stats || !work)
        return GHSVD_EINVAL;
    if (!aligned256(work)) return GHSVD_EINVAL;
    if (lwork < bpj_bytes(n_atoms, r)) return GHSVD_ENOMEM;
    return run_bpj(n_atoms, r, T, Mt, Jt, piv, stats, static_cast<char *>(work),
                   static_cast<hipStream_t>(stream));
}

extern "C" size_t ghsvd_phase1_workspace_size(int n_atoms, int nl) {
    const int r = 2 * nl;
    if (n_atoms < 1 || nl < 1 || r > kBpjMaxR) return 0;
    return bpj_bytes(n_atoms, r) + align_up((size_t)n_atoms * r * r * sizeof(double2), 256) +
           align_up((size_t)n_atoms * r * sizeof(int), 256);
}

extern "C" int ghsvd_phase1(int n_atoms, int nl, int n, const double *T, const double *H, int ldh,
                            const double *U, double *F, int ldf, signed char *J, double *G,
                            int ldg, int *stats, void *work, size_t lwork, void *stream) {
    const int r = 2 * nl;
    if (n_atoms < 1 || nl < 1 || r > kBpjMaxR || n < 1) return GHSVD_EINVAL;
    const long m = (long)r * n_atoms;
    if (!T || !H || !U || !F || !J || !G || !stats || !work) return GHSVD_EINVAL;
    if (ldh < m || ldf < m || ldg < m) return GHSVD_EINVAL;
    if (!aligned256(work)) return GHSVD_EINVAL;
    const size_t need = ghsvd_phase1_workspace_size(n_atoms, nl);
    if (lwork < need) return GHSVD_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(work);
    Carver c{w + bpj_bytes(n_atoms, r), 0, need - bpj_bytes(n_atoms, r)};
    double2 *Mt = c.take<double2>((size_t)n_atoms * r * r);
    int *piv = c.take<int>((size_t)n_atoms * r);
    const int rc = run_bpj(n_atoms, r, T, reinterpret_cast<double *>(Mt), J, piv, stats, w, st);
    if (rc != GHSVD_OK) return rc;
    const int nrt = (r + kApTile - 1) / kApTile, nct = (n + kApTile - 1) / kApTile;
    hipLaunchKernelGGL(k_p1_apply, dim3(nrt * nct, n_atoms), dim3(256), 0, st, r, nl, n, Mt,
                       reinterpret_cast<const double2 *>(H), ldh, U,
                       reinterpret_cast<double2 *>(F), ldf, reinterpret_cast<double2 *>(G), ldg);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}
