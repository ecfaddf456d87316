// post.hip -- outputs of the sweeps (Section 6.1.7 and eq. (3.2)).
//
// For every column j of the converged factors: h_j = f_j^* J f_j,
// s_j = g_j^* g_j, lambda_j = h_j / s_j (the signed squared generalized
// hyperbolic singular value), x_j = z'_j / sqrt(s_j) (so X^* S X = I), rows
// of X moved back by the column permutation P2 of the reduction
// (Section 5: Z~ = P2 Z), and, when asked, ascending order of lambda with the
// columns of X permuted alike (stable: ties keep the column order).
#include "post.hpp"

namespace ghsvd {

__global__ __launch_bounds__(256) void k_post_cols(int m, int nplus_unused, int p, int n,
                                                   const double2 *F, long ldf, const double2 *G,
                                                   long ldg, const double2 *Z, long ldz,
                                                   const double *gnorm2, double *lam,
                                                   double *scale, int *flags,
                                                   const int *nplus_dev) {
    __shared__ double red[3 * 256 / kWave];
    (void)nplus_unused;
    const int nplus = nplus_dev[0];
    const int j = blockIdx.x;
    const double2 *f = F + (size_t)j * ldf;
    const double2 *g = G + (size_t)j * ldg;
    const double2 *z = Z + (size_t)j * ldz;
    double v[3] = {0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < m; r += blockDim.x) v[0] += (r < nplus ? 1.0 : -1.0) * cnorm2(f[r]);
    for (int r = threadIdx.x; r < p; r += blockDim.x) v[1] += cnorm2(g[r]);
    for (int r = threadIdx.x; r < n; r += blockDim.x) v[2] += cnorm2(z[r]);
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        const double s = v[1];
        lam[j] = v[0] / s;
        scale[j] = 1.0 / sqrt(s);
        int bad = 0;
        if (!(s > 0.0)) bad |= 1;
        if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2])) bad |= 2;
        // G x_j has unit norm, so sigma_min(G) <= 1 / ||x_j||: numerical rank test.
        const double xn = sqrt(v[2] / s);
        if (!(xn * sqrt(gnorm2[0]) < 1.0 / (sqrt((double)n) * 0x1p-52))) bad |= 1;
        if (bad) atomicOr(flags, bad);
    }
}

__global__ void k_post_rank(int n, const double *lam, int *rank, int sort) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (!sort) {
        rank[j] = j;
        return;
    }
    const double lj = lam[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
        const double li = lam[i];
        r += (li < lj || (li == lj && i < j)) ? 1 : 0;
    }
    rank[j] = r;
}

__global__ void k_post_out(int n, const double2 *Z, long ldz, const double *lam, const double *scale,
                           const int *rank, const int *perm, double *lambda, double2 *X, long ldx) {
    const int j = blockIdx.y;
    const int col = rank[j];
    const double sc = scale[j];
    const double2 *z = Z + (size_t)j * ldz;
    double2 *x = X + (size_t)col * ldx;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int dst = perm ? perm[r] : r;
        x[dst] = cscale(z[r], sc);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) lambda[col] = lam[j];
}

// lambda[rank_j] = h_j / s_j, X(perm[i], rank_j) = Z(i, j) / sqrt(s_j);
// small[2] |= 1 when G is numerically rank deficient (a vanishing s_j, or
// ||x_j|| ||G||_F >= 1 / (sqrt(n) eps)), |= 2 for non-finite values.
int postprocess(const PencilDev &P, int sort, hipStream_t stream) {
    const int n = P.n;
    hipLaunchKernelGGL(k_post_cols, dim3(n), dim3(256), 0, stream, P.mr, 0, P.pr, n, P.Fw, P.ldf,
                       P.Gw, P.ldg, P.Zw, P.ldz, P.gnorm2, P.lam_tmp, P.scale, P.small + 2,
                       P.small + 1);
    hipLaunchKernelGGL(k_post_rank, dim3((n + 255) / 256), dim3(256), 0, stream, n, P.lam_tmp,
                       P.rank, sort);
    int bx = (n + 255) / 256;
    if (bx > 16) bx = 16;
    hipLaunchKernelGGL(k_post_out, dim3(bx, n), dim3(256), 0, stream, n, P.Zw, P.ldz, P.lam_tmp,
                       P.scale, P.rank, P.reduce ? P.perm : nullptr, P.lambda, P.X, P.ldx);
    GHSVD_HIP(hipGetLastError());
    return GHSVD_OK;
}

}  // namespace ghsvd
