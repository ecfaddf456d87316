// hz_step.hpp -- the FP64 2x2 Hari-Zimmermann transformation (Section 6.1).
//
// Given the pivot entries of (6.1) for columns p < q,
//   a = f_p^* J f_p, b = f_q^* J f_q, c = f_p^* J f_q,
//   sa = g_p^* g_p,  sb = g_q^* g_q,  sc = g_p^* g_q,
// computes Z' = D0 Z with Z the closed form (6.9)-(6.11) (phases removed by
// Phi_4), so that Z'^* S_hat Z' = I and Z'^* H_hat Z' is diagonal.
// Always evaluated in FP64, also when the columns are stored in FP32.
#pragma once

#include "hz_common.hpp"

namespace ghsvd {

enum : int { kSkip = 0, kSmall = 1, kBig = 2 };

// Arithmetic policies of the 2x2 step.  IeeeMath: correctly rounded division
// and square root (host and device).  FastMath (device): the hardware
// reciprocal / reciprocal square root refined by Newton steps (Markstein's
// formulation), about one ulp, for the latency-bound inner sweeps of the
// blocked variant; inputs are finite, positive where a root is taken, and
// far from the overflow and underflow thresholds.
struct IeeeMath {
    __host__ __device__ static double div(double a, double b) { return a / b; }
    __host__ __device__ static double sqrt_(double x) { return sqrt(x); }
    __host__ __device__ static double rsqrt(double x) { return 1.0 / sqrt(x); }
    __host__ __device__ static double hypot_(double a, double b) { return hypot(a, b); }
};

struct FastMath {
    __device__ static double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
        e = fma(-x, r, 1.0);
        return fma(r, e, r);
    }
    __device__ static double div(double a, double b) {
        const double r = rcp(b);
        const double q = a * r;
        return fma(fma(-b, q, a), r, q);
    }
    // returns (sqrt(x), 1 / sqrt(x)) for x > 0
    __device__ static void roots(double x, double &s, double &rs) {
        double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        r = fma(-g, g, x);
        s = fma(r, h, g);
        rs = 2.0 * h;
    }
    __device__ static double sqrt_(double x) {
        if (!(x > 0.0)) return x == 0.0 ? 0.0 : sqrt(x);
        double s, rs;
        roots(x, s, rs);
        return s;
    }
    // 1/sqrt(x) for x > 0: the hardware estimate (about 2^-24 relative) and
    // one third-order correction, y (1 - e)^(-1/2) ~ y (1 + e/2 + 3 e^2/8)
    // with e = 1 - x y^2, whose truncation error is near 2^-72; the result is
    // within about one ulp, four dependent operations after the estimate.
    __device__ static double rsqrt(double x) {
        const double y = __builtin_amdgcn_rsq(x);
        const double e = fma(-x * y, y, 1.0);
        return fma(y * e, fma(e, 0.375, 0.5), y);
    }
    __device__ static double hypot_(double a, double b) { return sqrt_(fma(a, a, b * b)); }
};

struct Zp {
    double2 z11, z21, z12, z22;  // column update: x_p' = x_p z11 + x_q z21, x_q' = x_p z12 + x_q z22
};

// Returns kSkip (no transformation: criterion (6.12) not met, or both
// off-diagonals exactly zero, Section 6.1.6), kSmall / kBig (cos phi = cos psi
// = 1 or not, Section 6.1.7), GHSVD_ERANK (G pair numerically dependent) or
// GHSVD_ENONFINITE.  Readings: sqrt form of (6.12) unless crit_literal;
// sigma = +1 at h = 0; the prescaled entries enter (6.4)-(6.12).
// f32_big = 1 classifies "big" with cos phi and cos psi rounded to FP32 (the
// FP32 warm-up stage).
template <class M>
__host__ __device__ inline int hz_step_m(double a, double b, double2 c, double sa, double sb,
                                         double2 sc, double tol, int crit_literal, Zp &z,
                                         int f32_big) {
    z.z11 = cmk(1.0, 0.0);
    z.z21 = cmk(0.0, 0.0);
    z.z12 = cmk(0.0, 0.0);
    z.z22 = cmk(1.0, 0.0);
    if (!isfinite(a) || !isfinite(b) || !isfinite(c.x) || !isfinite(c.y) || !isfinite(sa) ||
        !isfinite(sb) || !isfinite(sc.x) || !isfinite(sc.y))
        return GHSVD_ENONFINITE;
    if (!(sa > 0.0) || !(sb > 0.0)) return GHSVD_ERANK;

    // D0 prescaling (Section 6.1.1), applied per pivot pair.
    const double dp = M::rsqrt(sa);
    const double dq = M::rsqrt(sb);
    const double dpq = dp * dq;
    const double hpp = a * dp * dp;
    const double hqq = b * dq * dq;
    const double2 hpq = cscale(c, dpq);
    const double2 spq = cscale(sc, dpq);

    if (hpq.x == 0.0 && hpq.y == 0.0 && spq.x == 0.0 && spq.y == 0.0) return kSkip;

    const double habs = M::sqrt_(cnorm2(hpq));
    const double x = M::sqrt_(cnorm2(spq));
    const double ahp = fabs(hpp), ahq = fabs(hqq);
    const double thr = crit_literal ? (fmax(ahp, ahq) * tol) * fmin(ahp, ahq)
                                    : tol * M::sqrt_(ahp) * M::sqrt_(ahq);
    if (!(habs >= thr || x >= tol)) return kSkip;

    // Step 1: exp(i alpha_1) = s_pq / |s_pq| (1 when s_pq = 0), S1 = diag(1+x, 1-x).
    double2 e1 = cmk(1.0, 0.0);
    if (x > 0.0) {
        const double rx = M::div(1.0, x);
        e1 = cscale(spq, rx);
    }
    if (!(x < 1.0)) return GHSVD_ERANK;
    const double t = M::sqrt_((1.0 - x) * (1.0 + x));
    if (!(t > 0.0)) return GHSVD_ERANK;

    // Step 2: u + i v = conj(e1) h_pq.
    const double2 uv = cmulc(e1, hpq);
    const double u = uv.x, v = uv.y;
    const double h = hqq - hpp;

    int kind;
    double2 w11, w21, w12, w22;
    if (h == 0.0 && v == 0.0) {
        // Z = R1 D2 (Section 6.1.6).
        const double s2 = 0.70710678118654752440;
        const double d1 = s2 * M::rsqrt(1.0 + x);
        const double d2 = s2 * M::rsqrt(1.0 - x);
        w11 = cmk(d1, 0.0);
        w21 = cmk(e1.x * d1, -e1.y * d1);
        w12 = cmk(-e1.x * d2, -e1.y * d2);
        w22 = cmk(d2, 0.0);
        kind = kBig;
    } else {
        // Step 3 via (6.7) and (6.11), no trigonometric calls.
        const double sigma = (h >= 0.0) ? 1.0 : -1.0;
        const double twov = 2.0 * v;
        const double r = M::hypot_(h, twov);
        const double cos_g = M::div(fabs(h), r);
        const double sin_g = M::div(sigma * twov, r);
        const double num = sigma * (2.0 * u - (hpp + hqq) * x);
        const double den = t * r;
        const double rho = M::hypot_(num, den);
        const double cos_2t = M::div(den, rho);
        const double sin_2t = M::div(num, rho);
        // (6.10)
        const double base = 1.0 + t * cos_g * cos_2t;
        const double cphi = M::sqrt_(0.5 * (base + x * sin_2t));
        const double cpsi = M::sqrt_(0.5 * (base - x * sin_2t));
        const double im = t * sin_g * cos_2t;
        // e^{i alpha} sin(phi) = e1 ((sin2t - x) + i im) / (2 cos psi)
        const double ka = M::div(0.5, cpsi);
        const double2 ea = cmul(e1, cmk((sin_2t - x) * ka, im * ka));
        // e^{-i beta} sin(psi) = conj(e1) ((sin2t + x) - i im) / (2 cos phi)
        const double kb = M::div(0.5, cphi);
        const double2 eb = cmul(cconj(e1), cmk((sin_2t + x) * kb, -im * kb));
        const double rt = M::div(1.0, t);
        w11 = cmk(cphi * rt, 0.0);
        w12 = cscale(ea, rt);
        w21 = cscale(eb, -rt);
        w22 = cmk(cpsi * rt, 0.0);
        if (f32_big)
            kind = ((float)cphi == 1.0f && (float)cpsi == 1.0f) ? kSmall : kBig;
        else
            kind = (cphi == 1.0 && cpsi == 1.0) ? kSmall : kBig;
    }
    // Z' = D0 Z: row 1 scaled by d_p, row 2 by d_q.
    z.z11 = cscale(w11, dp);
    z.z12 = cscale(w12, dp);
    z.z21 = cscale(w21, dq);
    z.z22 = cscale(w22, dq);
    return kind;
}

__host__ __device__ inline int hz_step(double a, double b, double2 c, double sa, double sb,
                                       double2 sc, double tol, int crit_literal, Zp &z,
                                       int f32_big = 0) {
    return hz_step_m<IeeeMath>(a, b, c, sa, sb, sc, tol, crit_literal, z, f32_big);
}

// The 2x2 step for the latency-bound inner sweeps: the same closed form with
// FastMath roots, arranged so that the dependency chain holds four levels of
// reciprocal square roots instead of six.  1/sqrt(s_a), 1/sqrt(s_b) and
// 1/|s_c| are independent; they give x = |s_pq| = |s_c| d_p d_q, the phase
// e^{i alpha_1} = s_c / |s_c| and with it the pair (u, v) of (6.5), all
// without a root of x.  t = sqrt(1 - x^2) and r = sqrt(h^2 + 4 v^2) are then
// independent, rho follows from both, and cos phi, cos psi come last.
// "Small" (Section 6.1.7) is cos phi, cos psi within 2^-52 of 1, the
// resolution of a ~1-ulp root; f32_big classifies after rounding to FP32.
// Non-finite entries are not screened here: they propagate into the columns,
// where the FP64 pointwise sweeps that follow report them.
__device__ inline int hz_step_fast(double a, double b, double2 c, double sa, double sb,
                                   double2 sc, double tol, int crit_literal, Zp &z,
                                   int f32_big) {
    z.z11 = cmk(1.0, 0.0);
    z.z21 = cmk(0.0, 0.0);
    z.z12 = cmk(0.0, 0.0);
    z.z22 = cmk(1.0, 0.0);
    if (!(sa > 0.0) || !(sb > 0.0)) return GHSVD_ERANK;
    const double sc2 = cnorm2(sc);
    // level 1: three independent reciprocal roots
    const double dp = FastMath::rsqrt(sa);
    const double dq = FastMath::rsqrt(sb);
    const double rsc = sc2 > 0.0 ? FastMath::rsqrt(sc2) : 0.0;
    const double dpq = dp * dq;
    const double hpp = a * dp * dp;
    const double hqq = b * dq * dq;
    const double2 hpq = cscale(c, dpq);
    const double h2 = cnorm2(hpq);
    const double x = sc2 * rsc * dpq;  // |s_pq|
    const double x2 = x * x;
    if (h2 == 0.0 && x2 == 0.0) return kSkip;
    const double ahp = fabs(hpp), ahq = fabs(hqq);
    double thr2;
    if (crit_literal) {
        const double t1 = (fmax(ahp, ahq) * tol) * fmin(ahp, ahq);
        thr2 = t1 * t1;
    } else {
        thr2 = (tol * tol) * (ahp * ahq);
    }
    if (!(h2 >= thr2 || x2 >= tol * tol)) return kSkip;
    if (!(x < 1.0)) return GHSVD_ERANK;
    const double2 e1 = sc2 > 0.0 ? cscale(sc, rsc) : cmk(1.0, 0.0);
    // u + i v = conj(e1) h_pq
    const double2 uv = cmulc(e1, hpq);
    const double u = uv.x, v = uv.y;
    const double h = hqq - hpp;
    const double t2 = (1.0 - x) * (1.0 + x);
    if (!(t2 > 0.0)) return GHSVD_ERANK;
    // level 2: t and r
    const double rt = FastMath::rsqrt(t2);
    const double t = t2 * rt;
    int kind;
    double2 w11, w21, w12, w22;
    if (h == 0.0 && v == 0.0) {
        const double s2 = 0.70710678118654752440;
        const double d1 = s2 * FastMath::rsqrt(1.0 + x);
        const double d2 = s2 * FastMath::rsqrt(1.0 - x);
        w11 = cmk(d1, 0.0);
        w21 = cmk(e1.x * d1, -e1.y * d1);
        w12 = cmk(-e1.x * d2, -e1.y * d2);
        w22 = cmk(d2, 0.0);
        kind = kBig;
    } else {
        const double sigma = (h >= 0.0) ? 1.0 : -1.0;
        const double twov = 2.0 * v;
        const double q2 = fma(h, h, twov * twov);
        const double ir = FastMath::rsqrt(q2);
        const double r = q2 * ir;
        const double cos_g = fabs(h) * ir;
        const double sin_g = sigma * twov * ir;
        const double num = sigma * (2.0 * u - (hpp + hqq) * x);
        const double den = t * r;
        // level 3: rho
        const double n2 = fma(num, num, den * den);
        const double irho = FastMath::rsqrt(n2);
        const double cos_2t = den * irho;
        const double sin_2t = num * irho;
        const double base = 1.0 + t * cos_g * cos_2t;
        const double ap = 0.5 * (base + x * sin_2t);
        const double am = 0.5 * (base - x * sin_2t);
        // level 4: cos phi, cos psi
        const double iphi = FastMath::rsqrt(ap);
        const double ipsi = FastMath::rsqrt(am);
        const double cphi = ap * iphi;
        const double cpsi = am * ipsi;
        const double im = t * sin_g * cos_2t;
        const double ka = 0.5 * ipsi;
        const double2 ea = cmul(e1, cmk((sin_2t - x) * ka, im * ka));
        const double kb = 0.5 * iphi;
        const double2 eb = cmul(cconj(e1), cmk((sin_2t + x) * kb, -im * kb));
        w11 = cmk(cphi * rt, 0.0);
        w12 = cscale(ea, rt);
        w21 = cscale(eb, -rt);
        w22 = cmk(cpsi * rt, 0.0);
        if (f32_big)
            kind = ((float)cphi == 1.0f && (float)cpsi == 1.0f) ? kSmall : kBig;
        else
            kind = (cphi >= 1.0 - 0x1p-52 && cpsi >= 1.0 - 0x1p-52) ? kSmall : kBig;
    }
    z.z11 = cscale(w11, dp);
    z.z12 = cscale(w12, dp);
    z.z21 = cscale(w21, dq);
    z.z22 = cscale(w22, dq);
    return kind;
}

}  // namespace ghsvd
