/*
 * hz_oracle.c -- TEST INFRASTRUCTURE, not part of the solver.
 *
 * A plain, serial, double-precision CPU reference for the implicit
 * Hari-Zimmermann generalized hyperbolic SVD (Singer, Di Napoli, Novakovic,
 * Caklovic, "The LAPW method with eigendecomposition based on the
 * Hari-Zimmermann generalized hyperbolic SVD", arXiv:1907.08560).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file's library.  It shares no code, header, table or constant
 * with the GPU library: everything here is written out from the paper's
 * definitions, step by step, with no blocking, fusion or reordering.
 * Build: gcc -O2 -ffp-contract=off (no fast-math), one thread, no BLAS.
 *
 * Storage: column-major, complex values as C99 `double complex`
 * (interleaved re, im), signatures as int8 entries +1 / -1.
 *
 * Readings where the paper is silent or ambiguous (each one is listed in the
 * design notes of the repository):
 *   R1  criterion (6.12) compares |h_pq| with eps*sqrt(n)*sqrt(|h_pp||h_qq|);
 *       the printed product form is available as crit_literal = 1.
 *   R2  eps = 2^-52 for double precision.
 *   R3  sigma = sgn(h) is taken as +1 at h = 0.
 *   R4  a sweep ends the iteration when it applied no "big" transformation
 *       (Section 6.1.7); stop_rule = 1 selects "no transformation at all".
 *       The inner level of a blocked run (the Full Block variant) stops on
 *       an inner sweep with no transformation at all, as Section 6.1.7 says
 *       of inner levels.
 *   R5  the D0-prescaled pivot entries enter (6.4)-(6.12).
 *   R6  h_pq = s_pq = 0 skips the pair before (6.12) is evaluated.
 *   R7  G is taken as numerically rank deficient (error -2) when a pivot has
 *       |s_pq| >= sqrt(s_pp s_qq) after rounding, a column of G vanishes, or
 *       an output column has ||x_j|| ||G||_F >= 1 / (sqrt(n) eps).
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Status values returned by this file (integers fixed by the public
 * interface of the solver: 0 ok, 1 not converged, -1 invalid argument,
 * -2 rank deficient, -3 non-finite value). */
enum { ORA_OK = 0, ORA_NOT_CONVERGED = 1, ORA_EINVAL = -1, ORA_ERANK = -2,
       ORA_ENONFINITE = -3 };

/* Planted-mistake switch: the test suite rebuilds this file with
 * -DORA_MUTANT=k to check that its pins catch each mistake.  0 = correct. */
#ifndef ORA_MUTANT
#define ORA_MUTANT 0
#endif

#define COL(A, ld, i, j) ((A)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

/* ------------------------------------------------------------------------ */
/* The 2x2 step, Section 6.1 (6.2)-(6.12).                                   */
/* ------------------------------------------------------------------------ */

/*
 * Input: the pivot entries of (6.1), before prescaling:
 *   a = f_p^* J f_p, b = f_q^* J f_q, c = f_p^* J f_q,
 *   sa = g_p^* g_p, sb = g_q^* g_q, sc = g_p^* g_q;
 * tol = eps * sqrt(n).
 * Output zp[0..3] = Z' = D0 Z (column-major: z11, z21, z12, z22) and the
 * return value: 0 = pair skipped (Z' is the identity), 1 = transformed,
 * "small", 2 = transformed, "big", < 0 = error.
 */
int ora_pair_params(double a, double b, double c_re, double c_im,
                    double sa, double sb, double sc_re, double sc_im,
                    double tol, int crit_literal, double *zout)
{
    const cplx c = c_re + I * c_im;
    const cplx sc = sc_re + I * sc_im;
    cplx z11 = 1.0, z21 = 0.0, z12 = 0.0, z22 = 1.0;
    int kind;

    for (int i = 0; i < 8; ++i) zout[i] = 0.0;
    zout[0] = 1.0;
    zout[6] = 1.0;

    if (!isfinite(a) || !isfinite(b) || !isfinite(c_re) || !isfinite(c_im) ||
        !isfinite(sa) || !isfinite(sb) || !isfinite(sc_re) || !isfinite(sc_im))
        return ORA_ENONFINITE;
    if (!(sa > 0.0) || !(sb > 0.0))
        return ORA_ERANK;

    /* Section 6.1.1: prescaling of the pivot pair by D0 = diag(s_pp^-1/2, s_qq^-1/2). */
#if ORA_MUTANT == 11
    const double dp = 1.0;
    const double dq = 1.0;
#else
    const double dp = 1.0 / sqrt(sa);
    const double dq = 1.0 / sqrt(sb);
#endif
    const double hpp = a * dp * dp;
    const double hqq = b * dq * dq;
    const cplx hpq = c * (dp * dq);
    const cplx spq = sc * (dp * dq);

    /* Section 6.1.6, first exceptional case: both pivot blocks already diagonal. */
    if (hpq == 0.0 && spq == 0.0)
        return 0;

    /* Criterion (6.12). */
    const double habs = cabs(hpq);
    const double x = cabs(spq);
    double thr;
    if (crit_literal)
        thr = (fmax(fabs(hpp), fabs(hqq)) * tol) * fmin(fabs(hpp), fabs(hqq));
    else
        thr = tol * sqrt(fabs(hpp)) * sqrt(fabs(hqq));
    if (!(habs >= thr || x >= tol))
        return 0;

    /* Section 6.1.2: R1 with phi_1 = -pi/4 and alpha_1 = arg(s_pq) gives
     * S1 = diag(1 + x, 1 - x), (6.3).  x = 0 takes alpha_1 = 0 (6.1.6). */
    const cplx e1 = (x > 0.0) ? spq / x : 1.0;
    if (!(x < 1.0))
        return ORA_ERANK;
    const double t = sqrt((1.0 - x) * (1.0 + x));
    if (!(t > 0.0))
        return ORA_ERANK;

    /* (6.5): u + i v = exp(-i alpha_1) h_pq;  h = h_qq - h_pp (6.6). */
    const cplx w = conj(e1) * hpq;
    const double u = creal(w);
    const double v = cimag(w);
    const double h = hqq - hpp;

    if (h == 0.0 && v == 0.0) {
        /* Section 6.1.6, last case: Z = R1 D2. */
        const double r2 = 1.0 / sqrt(2.0);
        const double d1 = 1.0 / sqrt(1.0 + x);
        const double d2 = 1.0 / sqrt(1.0 - x);
        z11 = r2 * d1;
        z21 = r2 * conj(e1) * d1;
        z12 = -r2 * e1 * d2;
        z22 = r2 * d2;
        kind = 2;
    } else {
        /* sigma = sgn(h), gamma in (-pi/2, pi/2] with tan(gamma) = 2v/h (6.11). */
#if ORA_MUTANT == 13
        const double sigma = 1.0;
#else
        const double sigma = (h >= 0.0) ? 1.0 : -1.0;
#endif
        const double r = hypot(h, 2.0 * v);
        const double cg = fabs(h) / r;
        const double sg = sigma * (2.0 * v) / r;
        /* (6.7): tan(2 theta) = sigma (2u - (h_pp + h_qq) x) / (t sqrt(h^2 + 4 v^2)). */
#if ORA_MUTANT == 1
        const double num = sigma * (2.0 * u + (hpp + hqq) * x);
#else
        const double num = sigma * (2.0 * u - (hpp + hqq) * x);
#endif
        const double den = t * r;
        const double rho = hypot(num, den);
        const double c2 = den / rho;
        const double s2 = num / rho;
        /* (6.10) */
        const double cphi = sqrt(0.5 * (1.0 + x * s2 + t * cg * c2));
#if ORA_MUTANT == 2
        const double cpsi = sqrt(0.5 * (1.0 + x * s2 + t * cg * c2));
#else
        const double cpsi = sqrt(0.5 * (1.0 - x * s2 + t * cg * c2));
#endif
        const cplx esphi = e1 * ((s2 - x) + I * (t * sg * c2)) / (2.0 * cpsi);
#if ORA_MUTANT == 3
        const cplx espsi = e1 * ((s2 + x) - I * (t * sg * c2)) / (2.0 * cphi);
#else
        const cplx espsi = conj(e1) * ((s2 + x) - I * (t * sg * c2)) / (2.0 * cphi);
#endif
        /* (6.9) with the phases removed by Phi_4: Z = (1/t) [[cos phi, e^{i alpha} sin phi],
         *                                                   [-e^{-i beta} sin psi, cos psi]]. */
        z11 = cphi / t;
        z21 = -espsi / t;
        z12 = esphi / t;
        z22 = cpsi / t;
        kind = (cphi == 1.0 && cpsi == 1.0) ? 1 : 2;
    }

    /* Z' = D0 Z (end of Section 6.1.5). */
#if ORA_MUTANT == 4
    z11 *= dp; z12 *= dq; z21 *= dp; z22 *= dq;
#else
    z11 *= dp; z12 *= dp; z21 *= dq; z22 *= dq;
#endif
    zout[0] = creal(z11); zout[1] = cimag(z11);
    zout[2] = creal(z21); zout[3] = cimag(z21);
    zout[4] = creal(z12); zout[5] = cimag(z12);
    zout[6] = creal(z22); zout[7] = cimag(z22);
    return kind;
}

/* ------------------------------------------------------------------------ */
/* Pivot orderings, Section 6.3.                                              */
/* ------------------------------------------------------------------------ */

/* Row-cyclic order (Algorithm 2, "all pairs p < q"): pair number k of a sweep. */
static void row_cyclic_pairs(int n, int *pp, int *qq)
{
    int k = 0;
    for (int p = 0; p < n - 1; ++p)
        for (int q = p + 1; q < n; ++q) {
            pp[k] = p;
            qq[k] = q;
            ++k;
        }
}

/*
 * A cyclic parallel strategy in the sense of Section 6.3: the round-robin
 * ("circle") tournament.  Let N = n rounded up to an even number.  Step
 * s = 0..N-2 pairs slot N-1 with s, and (s+k) mod (N-1) with (s-k) mod (N-1)
 * for k = 1..N/2-1.  Each pair is written with p < q; for odd n the pair that
 * meets index n (the bye, Section 6.3.2) is dropped.  Writes the pairs of all
 * steps in order and returns the number of steps; steps have N/2 slots and a
 * dropped pair leaves p = q = -1.
 */
int ora_round_robin(int n, int *pp, int *qq)
{
    const int N = (n % 2) ? n + 1 : n;
    const int slots = N / 2;
    if (N < 2)
        return 0;
    for (int s = 0; s < N - 1; ++s) {
        for (int k = 0; k < slots; ++k) {
            int i, j;
            if (k == 0) {
                i = N - 1;
                j = s;
            } else {
                i = (s + k) % (N - 1);
#if ORA_MUTANT == 10
                j = (s + k + 1) % (N - 1);
#else
                j = ((s - k) % (N - 1) + (N - 1)) % (N - 1);
#endif
            }
            int p = i < j ? i : j, q = i < j ? j : i;
            if (q >= n) { p = -1; q = -1; }
            pp[s * slots + k] = p;
            qq[s * slots + k] = q;
        }
    }
    return N - 1;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: pointwise implicit HZ G(H)SVD.                               */
/* ------------------------------------------------------------------------ */

/* One pivot pair: (6.1) in one pass over the rows, the 2x2 step, and the
 * in-place column update [x_p, x_q] <- [x_p, x_q] Z'. */
static int hz_pair(int m, int p, int n, cplx *F, int ldf, const signed char *J,
                   cplx *G, int ldg, cplx *Z, int ldz, int pc, int qc,
                   double tol, int crit_literal)
{
    double a = 0.0, b = 0.0, sa = 0.0, sb = 0.0;
    cplx c = 0.0, sc = 0.0;
    for (int i = 0; i < m; ++i) {
        const cplx fp = COL(F, ldf, i, pc), fq = COL(F, ldf, i, qc);
        const double ji = (double)J[i];
        a += ji * (creal(fp) * creal(fp) + cimag(fp) * cimag(fp));
        b += ji * (creal(fq) * creal(fq) + cimag(fq) * cimag(fq));
#if ORA_MUTANT == 5
        c += ji * (fp * conj(fq));
#else
        c += ji * (conj(fp) * fq);
#endif
    }
    for (int i = 0; i < p; ++i) {
        const cplx gp = COL(G, ldg, i, pc), gq = COL(G, ldg, i, qc);
        sa += creal(gp) * creal(gp) + cimag(gp) * cimag(gp);
        sb += creal(gq) * creal(gq) + cimag(gq) * cimag(gq);
        sc += conj(gp) * gq;
    }
    double zz[8];
    const int kind = ora_pair_params(a, b, creal(c), cimag(c), sa, sb, creal(sc),
                                     cimag(sc), tol, crit_literal, zz);
    if (kind <= 0)
        return kind;
    const cplx z11 = zz[0] + I * zz[1], z21 = zz[2] + I * zz[3];
    const cplx z12 = zz[4] + I * zz[5], z22 = zz[6] + I * zz[7];
    for (int i = 0; i < m; ++i) {
        const cplx xp = COL(F, ldf, i, pc), xq = COL(F, ldf, i, qc);
        COL(F, ldf, i, pc) = xp * z11 + xq * z21;
        COL(F, ldf, i, qc) = xp * z12 + xq * z22;
    }
    for (int i = 0; i < p; ++i) {
        const cplx xp = COL(G, ldg, i, pc), xq = COL(G, ldg, i, qc);
        COL(G, ldg, i, pc) = xp * z11 + xq * z21;
        COL(G, ldg, i, qc) = xp * z12 + xq * z22;
    }
    for (int i = 0; i < n; ++i) {
        const cplx xp = COL(Z, ldz, i, pc), xq = COL(Z, ldz, i, qc);
#if ORA_MUTANT == 6
        COL(Z, ldz, i, pc) = xp * z11 + xq * z12;
        COL(Z, ldz, i, qc) = xp * z21 + xq * z22;
#else
        COL(Z, ldz, i, pc) = xp * z11 + xq * z21;
        COL(Z, ldz, i, qc) = xp * z12 + xq * z22;
#endif
    }
    return kind;
}

/*
 * Sweeps of Algorithm 2 in place on F (m x n), G (p x n) and Z' (n x n; the
 * caller initializes it, normally to I).  order: 0 row-cyclic, 1 round-robin.
 * stop_rule: 0 stop after a sweep with no big transformation, 1 after a sweep
 * with no transformation.  eps: the machine precision of (6.12).
 * stats[0] = sweeps run, [1] pairs visited, [2] transformed, [3] big,
 * [4] big transformations in the last sweep.
 * Returns 0 (converged), 1 (max_sweeps reached) or an error.
 */
int ora_hz_run(int m, int n, int p, cplx *F, int ldf, const signed char *J,
               cplx *G, int ldg, cplx *Z, int ldz, int order, int max_sweeps,
               double eps, int crit_literal, int stop_rule, long long *stats)
{
    if (m < 1 || n < 1 || p < 1 || ldf < m || ldg < p || ldz < n || max_sweeps < 1)
        return ORA_EINVAL;
    for (int i = 0; i < 5; ++i) stats[i] = 0;
    const double tol = eps * sqrt((double)n);
    int npairs, steps = 0, slots = 0;
    int *pp, *qq;
    if (order == 0) {
        npairs = n * (n - 1) / 2;
        pp = malloc(sizeof(int) * (size_t)(npairs + 1));
        qq = malloc(sizeof(int) * (size_t)(npairs + 1));
        row_cyclic_pairs(n, pp, qq);
    } else {
        const int N = (n % 2) ? n + 1 : n;
        slots = N / 2;
        npairs = (N - 1) * slots;
        pp = malloc(sizeof(int) * (size_t)(npairs + 1));
        qq = malloc(sizeof(int) * (size_t)(npairs + 1));
        steps = ora_round_robin(n, pp, qq);
        (void)steps;
    }
    int status = ORA_NOT_CONVERGED;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        long long tr = 0, big = 0;
        for (int k = 0; k < npairs; ++k) {
            if (pp[k] < 0)
                continue;
            const int kind = hz_pair(m, p, n, F, ldf, J, G, ldg, Z, ldz, pp[k], qq[k],
                                     tol, crit_literal);
            stats[1]++;
            if (kind < 0) {
                status = kind;
                goto done;
            }
            if (kind > 0) tr++;
            if (kind == 2) big++;
        }
        stats[0] = sweep;
        stats[2] += tr;
        stats[3] += big;
        stats[4] = big;
        if ((stop_rule == 0 && big == 0) || (stop_rule == 1 && tr == 0)) {
            status = ORA_OK;
            break;
        }
    }
done:
    free(pp);
    free(qq);
    return status;
}

/*
 * Outputs (Section 6.1.7 and Section 3): h_j = f_j^* J f_j, s_j = g_j^* g_j of
 * the final columns, lambda_j = h_j / s_j (the signed squared generalized
 * hyperbolic singular value, eq. (3.2)), X(:, j) = Z'(:, j) / sqrt(s_j), so
 * that X^* S X = I and X^* H X = diag(lambda).  sort = 1: ascending lambda
 * with X's columns permuted alike (ties keep the column order).
 */
int ora_hz_post(int m, int n, int p, const cplx *F, int ldf, const signed char *J,
                const cplx *G, int ldg, const cplx *Z, int ldz, int sort,
                double *lambda, cplx *X, int ldx)
{
    double *lam = malloc(sizeof(double) * (size_t)n);
    double *sn = malloc(sizeof(double) * (size_t)n);
    int *idx = malloc(sizeof(int) * (size_t)n);
    int status = ORA_OK;
    for (int j = 0; j < n; ++j) {
        double h = 0.0, s = 0.0;
        for (int i = 0; i < m; ++i) {
            const cplx f = COL(F, ldf, i, j);
            h += (double)J[i] * (creal(f) * creal(f) + cimag(f) * cimag(f));
        }
        for (int i = 0; i < p; ++i) {
            const cplx g = COL(G, ldg, i, j);
            s += creal(g) * creal(g) + cimag(g) * cimag(g);
        }
        if (!(s > 0.0)) status = ORA_ERANK;
        lam[j] = h / s;
        sn[j] = sqrt(s);
        idx[j] = j;
    }
    if (sort) { /* insertion sort: stable, plain */
        for (int j = 1; j < n; ++j) {
            const int t = idx[j];
            int k = j - 1;
            while (k >= 0 && lam[idx[k]] > lam[t]) {
                idx[k + 1] = idx[k];
                --k;
            }
            idx[k + 1] = t;
        }
    }
    for (int j = 0; j < n; ++j) {
        const int src = idx[j];
        lambda[j] = lam[src];
        for (int i = 0; i < n; ++i)
#if ORA_MUTANT == 9
            COL(X, ldx, i, j) = COL(Z, ldz, i, src) * sn[src];
#else
            COL(X, ldx, i, j) = COL(Z, ldz, i, src) / sn[src];
#endif
    }
    free(lam);
    free(sn);
    free(idx);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Section 5: one-time reduction to square factors.                          */
/* ------------------------------------------------------------------------ */

/*
 * Householder QR of A (p x n, p >= n) in place: on return the upper triangle
 * holds R and the rest is zero.  Convention: R_kk = -e^{i arg x_1} ||x|| for
 * the column x being reduced (e^{i arg 0} = 1), so R is unique.
 */
int ora_qr(int p, int n, cplx *A, int lda)
{
    if (p < n || lda < p) return ORA_EINVAL;
    cplx *v = malloc(sizeof(cplx) * (size_t)p);
    for (int k = 0; k < n; ++k) {
        double nrm2 = 0.0;
        for (int i = k; i < p; ++i) {
            const cplx x = COL(A, lda, i, k);
            nrm2 += creal(x) * creal(x) + cimag(x) * cimag(x);
        }
        const double nrm = sqrt(nrm2);
        if (nrm == 0.0) continue;
        const cplx x1 = COL(A, lda, k, k);
        const double ax1 = cabs(x1);
        const cplx ph = (ax1 > 0.0) ? x1 / ax1 : 1.0;
        const cplx beta = -ph * nrm;
        for (int i = k; i < p; ++i) v[i] = COL(A, lda, i, k);
#if ORA_MUTANT == 7
        v[k] = ph * (ax1 - nrm);
#else
        v[k] = ph * (ax1 + nrm);
#endif
        const double vv = 2.0 * nrm * (nrm + ax1); /* v^* v */
        for (int j = k + 1; j < n; ++j) {
            cplx w = 0.0;
            for (int i = k; i < p; ++i) w += conj(v[i]) * COL(A, lda, i, j);
            w *= 2.0 / vv;
            for (int i = k; i < p; ++i) COL(A, lda, i, j) -= v[i] * w;
        }
        COL(A, lda, k, k) = beta;
        for (int i = k + 1; i < p; ++i) COL(A, lda, i, k) = 0.0;
    }
    free(v);
    return ORA_OK;
}

static double jnorm2(const cplx *A, int lda, const signed char *J, int r0, int m, int c)
{
    double h = 0.0;
    for (int i = r0; i < m; ++i) {
        const cplx f = COL(A, lda, i, c);
        h += (double)J[i] * (creal(f) * creal(f) + cimag(f) * cimag(f));
    }
    return h;
}

static cplx jdot(const cplx *A, int lda, const signed char *J, int r0, int m, int c1, int c2)
{
    cplx s = 0.0;
    for (int i = r0; i < m; ++i)
        s += (double)J[i] * (conj(COL(A, lda, i, c1)) * COL(A, lda, i, c2));
    return s;
}

static void swap_cols(cplx *A, int lda, int m, int c1, int c2, int *perm)
{
    if (c1 == c2) return;
    for (int i = 0; i < m; ++i) {
        const cplx t = COL(A, lda, i, c1);
        COL(A, lda, i, c1) = COL(A, lda, i, c2);
        COL(A, lda, i, c2) = t;
    }
    const int t = perm[c1];
    perm[c1] = perm[c2];
    perm[c2] = t;
}

/*
 * Hyperbolic Householder reflector (Theorem 5.1 and Section 5.3) that maps
 * column c, rows r0..m-1, to -c_1 e_1 with |c_1| = |f^* J f|^(1/2) and
 * arg c_1 = arg f_11, using the generator s = f + c_1 e_1 and
 * tau = -1 / (f^* J f + |f^* J f|^(1/2) |f_11| j_11).  If the sign of j_11
 * does not match that of f^* J f, the matching-sign row holding the largest
 * |f_i| is swapped to the front first (whole rows, with J).  The reflector
 * is applied to columns c+1..n-1.
 */
static int hyp_reflect(int m, int n, cplx *A, int lda, signed char *J, int r0, int c, cplx *s)
{
    const double h = jnorm2(A, lda, J, r0, m, c);
    if (!isfinite(h)) return ORA_ENONFINITE;
    if (h == 0.0) return ORA_ERANK;
    const signed char sg = (h > 0.0) ? 1 : -1;
    if (J[r0] != sg) {
        int best = -1;
        double bv = -1.0;
        for (int i = r0; i < m; ++i)
            if (J[i] == sg && cabs(COL(A, lda, i, c)) > bv) {
                bv = cabs(COL(A, lda, i, c));
                best = i;
            }
        if (best < 0) return ORA_ERANK;
        for (int j = 0; j < n; ++j) {
            const cplx t = COL(A, lda, r0, j);
            COL(A, lda, r0, j) = COL(A, lda, best, j);
            COL(A, lda, best, j) = t;
        }
        J[best] = J[r0];
        J[r0] = sg;
    }
    const cplx f11 = COL(A, lda, r0, c);
    const double af = cabs(f11);
    const cplx e = (af > 0.0) ? f11 / af : 1.0;
    const double r = sqrt(fabs(h));
    const cplx c1 = r * e;
    for (int i = r0; i < m; ++i) s[i] = COL(A, lda, i, c);
    s[r0] = e * (af + r);
    const double tau = -1.0 / (h + r * af * (double)J[r0]);
    for (int j = c + 1; j < n; ++j) {
        cplx w = 0.0;
#if ORA_MUTANT == 8
        for (int i = r0; i < m; ++i) w += conj(s[i]) * COL(A, lda, i, j);
#else
        for (int i = r0; i < m; ++i) w += conj(s[i]) * ((double)J[i] * COL(A, lda, i, j));
#endif
        w *= tau;
        for (int i = r0; i < m; ++i) COL(A, lda, i, j) += s[i] * w;
    }
    COL(A, lda, r0, c) = -c1;
    for (int i = r0 + 1; i < m; ++i) COL(A, lda, i, c) = 0.0;
    return ORA_OK;
}

/*
 * JQR of A (m x n) under J (Section 5, eq. (5.1)), with the column pivoting
 * of Section 5.2.1 (diagonal pivoting plus Bunch-Kaufman partial pivoting,
 * alpha = (1 + sqrt(17)) / 8), single pivots by the hyperbolic reflector of
 * Section 5.3, and 2x2 pivots by the (J, I) URV scheme: a Jacobi rotation R
 * of the pivot J-Gram, two reflectors, then R^* on the pivot columns.
 * On return A[0..n-1, 0..n-1] is the block upper triangular square factor,
 * the rows below are zero, J[0..n-1] is its signature, perm[i] is the input
 * column now at position i (P2), and *n2x2 counts the 2x2 pivots.
 */
int ora_jqr(int m, int n, cplx *A, int lda, signed char *J, int *perm, int *n2x2)
{
    if (m < n || lda < m) return ORA_EINVAL;
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    double *hd = malloc(sizeof(double) * (size_t)n);
    cplx *s = malloc(sizeof(cplx) * (size_t)m);
    int status = ORA_OK;
    for (int j = 0; j < n; ++j) perm[j] = j;
    *n2x2 = 0;
    int k = 0;
    while (k < n) {
        /* Diagonal pivoting: the largest |h_ii| of the trailing J_k-Gram. */
        for (int i = k; i < n; ++i) hd[i] = jnorm2(A, lda, J, k, m, i);
        int jmax = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(hd[i]) > fabs(hd[jmax])) jmax = i;
        if (jmax != k) {
            swap_cols(A, lda, m, k, jmax, perm);
            const double t = hd[k]; hd[k] = hd[jmax]; hd[jmax] = t;
        }
        int piv = 1;
        if (k < n - 1) {
            /* Partial pivoting (Bunch-Kaufman Algorithm C) on row 1 of H_k. */
            int ii = k + 1;
            double lam = -1.0;
            for (int j = k + 1; j < n; ++j) {
                const double v = cabs(jdot(A, lda, J, k, m, k, j));
                if (v > lam) { lam = v; ii = j; }
            }
#if ORA_MUTANT == 14
            if (0) {
#else
            if (!(fabs(hd[k]) >= alpha * lam)) {
#endif
                double sig = -1.0;
                for (int l = k; l < n; ++l) {
                    if (l == ii) continue;
                    const double v = cabs(jdot(A, lda, J, k, m, ii, l));
                    if (v > sig) sig = v;
                }
                if (fabs(hd[k]) * sig >= alpha * lam * lam) {
                    piv = 1;
                } else if (fabs(hd[ii]) >= alpha * sig) {
                    swap_cols(A, lda, m, k, ii, perm);
                    const double t = hd[k]; hd[k] = hd[ii]; hd[ii] = t;
                    piv = 1;
                } else {
                    piv = 2;
                    if (ii != k + 1) {
                        swap_cols(A, lda, m, k + 1, ii, perm);
                        const double t = hd[k + 1]; hd[k + 1] = hd[ii]; hd[ii] = t;
                    }
                }
            }
        }
        if (piv == 1) {
            status = hyp_reflect(m, n, A, lda, J, k, k, s);
            if (status != ORA_OK) break;
            k += 1;
        } else {
            /* (J, I) URV step on the pivot block [f_k, f_k+1]. */
            const double h11 = jnorm2(A, lda, J, k, m, k);
            const double h22 = jnorm2(A, lda, J, k, m, k + 1);
            const cplx h12 = jdot(A, lda, J, k, m, k, k + 1);
            double co = 1.0, si = 0.0;
            cplx eph = 1.0;
            const double ah = cabs(h12);
            if (ah > 0.0) {
                /* Jacobi rotation R = [[co, e si], [-conj(e) si, co]], e = h12/|h12|,
                 * tan(2 theta) = 2|h12| / (h22 - h11), |theta| <= pi/4. */
                eph = h12 / ah;
                const double tt = (h22 - h11) / (2.0 * ah);
                const double tn = (tt >= 0.0 ? 1.0 : -1.0) / (fabs(tt) + sqrt(1.0 + tt * tt));
                co = 1.0 / sqrt(1.0 + tn * tn);
                si = tn * co;
            }
            for (int i = k; i < m; ++i) {
                const cplx x1 = COL(A, lda, i, k), x2 = COL(A, lda, i, k + 1);
                COL(A, lda, i, k) = co * x1 - conj(eph) * si * x2;
                COL(A, lda, i, k + 1) = eph * si * x1 + co * x2;
            }
            status = hyp_reflect(m, n, A, lda, J, k, k, s);
            if (status != ORA_OK) break;
            status = hyp_reflect(m, n, A, lda, J, k + 1, k + 1, s);
            if (status != ORA_OK) break;
            /* Multiply the (now 2-row) pivot block by R^*. */
            for (int i = k; i < k + 2; ++i) {
                const cplx x1 = COL(A, lda, i, k), x2 = COL(A, lda, i, k + 1);
                COL(A, lda, i, k) = co * x1 + conj(eph) * si * x2;
                COL(A, lda, i, k + 1) = -eph * si * x1 + co * x2;
            }
            *n2x2 += 1;
            k += 2;
        }
    }
    free(hd);
    free(s);
    return status;
}

/*
 * The whole path on the CPU: optional reduction (JQR of F with P2, QR of
 * G P2, Section 5), sweeps of Algorithm 2, the outputs of Section 6.1.7,
 * and the row permutation of the eigenvectors back by P2 (Z~ = P2 Z).
 * Inputs are not modified.  stats as in ora_hz_run; stats[5] = 2x2 pivots.
 * X (n x n) satisfies F^* J F X = G^* G X diag(lambda), X^* G^* G X = I.
 */
int ora_ghsvd(int m, int n, int p, const cplx *F, int ldf, const signed char *J,
              const cplx *G, int ldg, int reduce, int order, int max_sweeps,
              double eps, int crit_literal, int sort, double *lambda, cplx *X, int ldx,
              long long *stats)
{
    if (m < n || p < n || n < 1 || ldf < m || ldg < p || ldx < n) return ORA_EINVAL;
    for (int i = 0; i < 6; ++i) stats[i] = 0;
    int status;
    int mr = m, pr = p;
    cplx *Fw, *Gw;
    signed char *Jw = malloc((size_t)m);
    int *perm = malloc(sizeof(int) * (size_t)n);
    memcpy(Jw, J, (size_t)m);
    for (int j = 0; j < n; ++j) perm[j] = j;
    if (reduce) {
        cplx *Ft = malloc(sizeof(cplx) * (size_t)m * n);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) Ft[(size_t)j * m + i] = COL(F, ldf, i, j);
        int n2 = 0;
        status = ora_jqr(m, n, Ft, m, Jw, perm, &n2);
        stats[5] = n2;
        if (status != ORA_OK) { free(Ft); free(Jw); free(perm); return status; }
        cplx *Gt = malloc(sizeof(cplx) * (size_t)p * n);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < p; ++i) Gt[(size_t)j * p + i] = COL(G, ldg, i, perm[j]);
        status = ora_qr(p, n, Gt, p);
        mr = n;
        pr = n;
        Fw = malloc(sizeof(cplx) * (size_t)n * n);
        Gw = malloc(sizeof(cplx) * (size_t)n * n);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                Fw[(size_t)j * n + i] = Ft[(size_t)j * m + i];
                Gw[(size_t)j * n + i] = Gt[(size_t)j * p + i];
            }
        free(Ft);
        free(Gt);
    } else {
        Fw = malloc(sizeof(cplx) * (size_t)m * n);
        Gw = malloc(sizeof(cplx) * (size_t)p * n);
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < m; ++i) Fw[(size_t)j * m + i] = COL(F, ldf, i, j);
            for (int i = 0; i < p; ++i) Gw[(size_t)j * p + i] = COL(G, ldg, i, j);
        }
    }
    cplx *Zw = calloc((size_t)n * n, sizeof(cplx));
    for (int j = 0; j < n; ++j) Zw[(size_t)j * n + j] = 1.0;
    status = ora_hz_run(mr, n, pr, Fw, mr, Jw, Gw, pr, Zw, n, order, max_sweeps, eps,
                        crit_literal, 0, stats);
    if (status >= 0) {
        cplx *Xs = malloc(sizeof(cplx) * (size_t)n * n);
        const int ps = ora_hz_post(mr, n, pr, Fw, mr, Jw, Gw, pr, Zw, n, sort, lambda, Xs, n);
        if (ps != ORA_OK) status = ps;
        /* Numerical rank of G (reading R7): G x_j has unit norm, so
         * sigma_min(G) <= 1 / ||x_j||; flag ||x_j|| ||G||_F >= 1 / (sqrt(n) eps). */
        double gf = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < p; ++i) {
                const cplx g = COL(G, ldg, i, j);
                gf += creal(g) * creal(g) + cimag(g) * cimag(g);
            }
        gf = sqrt(gf);
        for (int j = 0; j < n && status >= 0; ++j) {
            double xn = 0.0;
            for (int i = 0; i < n; ++i) {
                const cplx x = Xs[(size_t)j * n + i];
                xn += creal(x) * creal(x) + cimag(x) * cimag(x);
            }
            if (!(sqrt(xn) * gf < 1.0 / (sqrt((double)n) * eps))) status = ORA_ERANK;
        }
        for (int j = 0; j < n; ++j)
#if ORA_MUTANT == 12
            for (int i = 0; i < n; ++i) COL(X, ldx, i, j) = Xs[(size_t)j * n + i];
#else
            for (int i = 0; i < n; ++i) COL(X, ldx, perm[i], j) = Xs[(size_t)j * n + i];
#endif
        free(Xs);
    }
    free(Fw);
    free(Gw);
    free(Zw);
    free(Jw);
    free(perm);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Section 6.4: Level-2 blocked sweeps, Block-Oriented (BO) inner level.     */
/* ------------------------------------------------------------------------ */

/*
 * Block columns of width w: block b holds columns [b w, min(b w + w, n)); the
 * number of blocks nb is ceil(n / w) rounded up to even (trailing blocks may
 * be narrow or empty).  A block step pairs blocks by the round-robin ordering
 * over nb; for a block pair (a, b) the pivot columns are those of a followed
 * by those of b (c of them).  The block pivot is shortened by the (J)QR
 * approach of Section 6.4.2: JQR of F_C under J gives F^ (c x c) with J^ and
 * P, QR of G_C P gives G^; with the columns put back in the pivot order
 * (F~ = F^ P^T, G~ = G^ P^T) they satisfy F~^* J^ F~ = F_C^* J F_C and
 * G~^* G~ = G_C^* G_C.  One inner sweep of Algorithm 2 (BO: C_max = 1, the
 * round-robin order over c) on (F~, J^, G~) accumulates Z^ (c x c), and, if
 * it transformed anything, F_C, G_C and Z_C are multiplied by Z^
 * (Section 6.4.3).  After each block sweep the iteration stops when the
 * inner sweeps applied no big transformation.  stats as ora_hz_run, counting
 * inner pivot pairs; stats[5] = the most inner sweeps any block pivot ran.
 * eps is the machine precision of (6.12) with n the order of the block pivot
 * (tol = eps sqrt(c)).
 *
 * inner_order 2 is the Full Block (FB) variant of Section 6.4.2: the inner
 * level runs round-robin sweeps over the c pivot columns until one of them
 * applies no transformation at all, big or small (Section 6.1.7: the inner
 * levels of a blocked algorithm count every transformation for stopping, as
 * Algorithm 2's own test does), at most C_max = 30 of them; Z^ accumulates
 * them all.  Only the outer level stops on the absence of big
 * transformations.  BO is the same with C_max = 1.
 *
 * inner_order 3 and 4 apply the blocking principle once more (Section 6.4:
 * the Level-2 principle applied recursively): the shortened block pivot
 * (F~, J^, G~), of order c, is itself swept by this Level-2 blocked run with
 * block width ORA_ML_WIDTH and its own BO inner level (inner_order 0), one
 * blocked sweep (3) or blocked sweeps until one applies no big
 * transformation, at most C_max = 30 (4); Z^ accumulates them.  The nested
 * run re-forms its own block pivots every sweep, so rounding keeps small
 * transformations coming and the "no transformation at all" test of a
 * pointwise inner level (Section 6.1.7) need not be met: it stops like an
 * outer level.  stats count the innermost pivot pairs; stats[5] = the most
 * nested blocked sweeps any block pivot ran.
 */
#define ORA_ML_WIDTH 8

static int block_run(int m, int n, int p, cplx *F, int ldf, const signed char *J, cplx *G,
                     int ldg, cplx *Z, int ldz, int w, int max_sweeps, double eps,
                     int crit_literal, int inner_order, int stop_all, long long *stats);

int ora_hz_block_run(int m, int n, int p, cplx *F, int ldf, const signed char *J,
                     cplx *G, int ldg, cplx *Z, int ldz, int w, int max_sweeps,
                     double eps, int crit_literal, int inner_order, long long *stats)
{
    if (inner_order < 0 || inner_order > 4) return ORA_EINVAL;
    return block_run(m, n, p, F, ldf, J, G, ldg, Z, ldz, w, max_sweeps, eps, crit_literal,
                     inner_order, 0, stats);
}

/* The same with the stopping test chosen: stop_all = 1 stops after a blocked
 * sweep with no transformation at all (the test of an inner level, Section
 * 6.1.7), 0 after one with no big transformation. */
int ora_hz_block_run_ex(int m, int n, int p, cplx *F, int ldf, const signed char *J,
                        cplx *G, int ldg, cplx *Z, int ldz, int w, int max_sweeps,
                        double eps, int crit_literal, int inner_order, int stop_all,
                        long long *stats)
{
    if (inner_order < 0 || inner_order > 4) return ORA_EINVAL;
    return block_run(m, n, p, F, ldf, J, G, ldg, Z, ldz, w, max_sweeps, eps, crit_literal,
                     inner_order, stop_all != 0, stats);
}

static int block_run(int m, int n, int p, cplx *F, int ldf, const signed char *J, cplx *G,
                     int ldg, cplx *Z, int ldz, int w, int max_sweeps, double eps,
                     int crit_literal, int inner_order, int stop_all, long long *stats)
{
    if (m < 1 || n < 2 || p < 1 || ldf < m || ldg < p || ldz < n || w < 1 || max_sweeps < 1)
        return ORA_EINVAL;
    for (int i = 0; i < 6; ++i) stats[i] = 0;
    int nb = (n + w - 1) / w;
    if (nb % 2) nb += 1;
    int bsteps = 0;
    int *bp = malloc(sizeof(int) * (size_t)nb * nb), *bq = malloc(sizeof(int) * (size_t)nb * nb);
    bsteps = ora_round_robin(nb, bp, bq);
    const int bslots = nb / 2;
    const int cmax = 2 * w;
    const int cneed = cmax < n ? cmax : n;  /* a block pivot's columns: m, p must cover them */
    if (m < cneed || p < cneed) { free(bp); free(bq); return ORA_EINVAL; }
    int *cols = malloc(sizeof(int) * (size_t)cmax);
    cplx *FC = malloc(sizeof(cplx) * (size_t)m * cmax);
    cplx *GC = malloc(sizeof(cplx) * (size_t)p * cmax);
    cplx *Ft = malloc(sizeof(cplx) * (size_t)cmax * cmax);
    cplx *Gt = malloc(sizeof(cplx) * (size_t)cmax * cmax);
    cplx *Zh = malloc(sizeof(cplx) * (size_t)cmax * cmax);
    cplx *tmp = malloc(sizeof(cplx) * (size_t)(m > p ? (m > n ? m : n) : (p > n ? p : n)) * cmax);
    signed char *Jw = malloc((size_t)m);
    int *perm = malloc(sizeof(int) * (size_t)cmax);
    int *ip = malloc(sizeof(int) * (size_t)cmax * cmax), *iq = malloc(sizeof(int) * (size_t)cmax * cmax);
    int status = ORA_NOT_CONVERGED;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        long long tr = 0, big = 0;
        for (int s = 0; s < bsteps; ++s) {
            for (int k = 0; k < bslots; ++k) {
                const int a = bp[s * bslots + k], b = bq[s * bslots + k];
                if (a < 0) continue;
                int c = 0;
                for (int j = a * w; j < a * w + w && j < n; ++j) cols[c++] = j;
                for (int j = b * w; j < b * w + w && j < n; ++j) cols[c++] = j;
                if (c < 2) continue;
                for (int j = 0; j < c; ++j) {
                    for (int i = 0; i < m; ++i) FC[(size_t)j * m + i] = COL(F, ldf, i, cols[j]);
                    for (int i = 0; i < p; ++i) GC[(size_t)j * p + i] = COL(G, ldg, i, cols[j]);
                }
                /* (J)QR shortening of the block pivot */
                memcpy(Jw, J, (size_t)m);
                int n2 = 0;
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < m; ++i) tmp[(size_t)j * m + i] = FC[(size_t)j * m + i];
                int st = ora_jqr(m, c, tmp, m, Jw, perm, &n2);
                if (st != ORA_OK) { status = st; goto done; }
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < c; ++i) Ft[(size_t)perm[j] * c + i] = tmp[(size_t)j * m + i];
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < p; ++i) tmp[(size_t)j * p + i] = GC[(size_t)perm[j] * p + i];
                st = ora_qr(p, c, tmp, p);
                if (st != ORA_OK) { status = st; goto done; }
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < c; ++i) Gt[(size_t)perm[j] * c + i] = tmp[(size_t)j * p + i];
                /* one inner sweep (BO): round-robin over the c pivot columns, or,
                 * with inner_order = 1 at every block step but the first of the
                 * sweep, only the w x w pairs across two full blocks: step k
                 * pairs column i of block a with column (i + k) mod w of block b.
                 * The first block step meets every block once, so then each
                 * pair of columns is visited once per sweep. */
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < c; ++i) Zh[(size_t)j * c + i] = (i == j) ? 1.0 : 0.0;
                if (inner_order >= 3) {
                    /* the shortened pivot swept by the Level-2 blocked run */
                    long long st2[6];
#if ORA_MUTANT == 16
                    const int wml = w;
#else
                    const int wml = ORA_ML_WIDTH;
#endif
                    const int rs = block_run(c, c, c, Ft, c, Jw, Gt, c, Zh, c, wml,
                                             inner_order == 4 ? 30 : 1, eps, crit_literal, 0, 0,
                                             st2);
                    if (rs < 0) { status = rs; goto done; }
                    stats[1] += st2[1];
                    tr += st2[2];
                    big += st2[3];
                    if (st2[0] > stats[5]) stats[5] = st2[0];
                    if (st2[2] == 0) continue;
                    goto update;
                }
                int isteps, islots;
                const int ca = (a * w + w <= n) ? w : (a * w < n ? n - a * w : 0);
                const int cmax_inner = inner_order == 2 ? 30 : 1;
                if (inner_order == 1 && s > 0 && ca == w && c == 2 * w) {
                    isteps = w;
                    islots = w;
                    for (int is = 0; is < w; ++is)
                        for (int ik = 0; ik < w; ++ik) {
                            ip[is * w + ik] = ik;
                            iq[is * w + ik] = w + (ik + is) % w;
                        }
                } else {
                    isteps = ora_round_robin(c, ip, iq);
                    islots = (c + (c % 2)) / 2;
                }
                const double tol = eps * sqrt((double)c);
                long long itr = 0;
                for (int isw = 0; isw < cmax_inner; ++isw) {
                    /* transformations (all, and big) of this inner sweep */
                    long long iall = 0, ibig = 0;
                    for (int is = 0; is < isteps; ++is)
                        for (int ik = 0; ik < islots; ++ik) {
                            const int pc = ip[is * islots + ik], qc = iq[is * islots + ik];
                            if (pc < 0) continue;
                            const int kind = hz_pair(c, c, c, Ft, c, Jw, Gt, c, Zh, c, pc, qc, tol,
                                                     crit_literal);
                            stats[1]++;
                            if (kind == ORA_ERANK) continue; /* left to the finishing sweeps */
                            if (kind < 0) { status = kind; goto done; }
                            if (kind > 0) { tr++; itr++; iall++; }
                            if (kind == 2) { big++; ibig++; }
                        }
                    if (isw + 1 > stats[5]) stats[5] = isw + 1;
#if ORA_MUTANT == 15
                    (void)iall;
                    if (ibig == 0) break;
#else
                    (void)ibig;
                    if (iall == 0) break;
#endif
                }
                if (itr == 0) continue;
            update:
                /* F_C <- F_C Z^, G_C <- G_C Z^, Z_C <- Z_C Z^ (Section 6.4.3) */
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < m; ++i) {
                        cplx acc = 0.0;
                        for (int l = 0; l < c; ++l) acc += FC[(size_t)l * m + i] * Zh[(size_t)j * c + l];
                        COL(F, ldf, i, cols[j]) = acc;
                    }
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < p; ++i) {
                        cplx acc = 0.0;
                        for (int l = 0; l < c; ++l) acc += GC[(size_t)l * p + i] * Zh[(size_t)j * c + l];
                        COL(G, ldg, i, cols[j]) = acc;
                    }
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < n; ++i) tmp[(size_t)j * n + i] = COL(Z, ldz, i, cols[j]);
                for (int j = 0; j < c; ++j)
                    for (int i = 0; i < n; ++i) {
                        cplx acc = 0.0;
                        for (int l = 0; l < c; ++l) acc += tmp[(size_t)l * n + i] * Zh[(size_t)j * c + l];
                        COL(Z, ldz, i, cols[j]) = acc;
                    }
            }
        }
        stats[0] = sweep;
        stats[2] += tr;
        stats[3] += big;
        stats[4] = big;
        if ((stop_all ? tr : big) == 0) { status = ORA_OK; break; }
    }
done:
    free(bp); free(bq); free(cols); free(FC); free(GC); free(Ft); free(Gt); free(Zh); free(tmp);
    free(Jw); free(perm); free(ip); free(iq);
    return status;
}
