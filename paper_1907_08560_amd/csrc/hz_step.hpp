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
__host__ __device__ inline int hz_step(double a, double b, double2 c, double sa, double sb,
                                       double2 sc, double tol, int crit_literal, Zp &z,
                                       int f32_big = 0) {
    z.z11 = cmk(1.0, 0.0);
    z.z21 = cmk(0.0, 0.0);
    z.z12 = cmk(0.0, 0.0);
    z.z22 = cmk(1.0, 0.0);
    if (!isfinite(a) || !isfinite(b) || !isfinite(c.x) || !isfinite(c.y) || !isfinite(sa) ||
        !isfinite(sb) || !isfinite(sc.x) || !isfinite(sc.y))
        return GHSVD_ENONFINITE;
    if (!(sa > 0.0) || !(sb > 0.0)) return GHSVD_ERANK;

    // D0 prescaling (Section 6.1.1), applied per pivot pair.
    const double dp = 1.0 / sqrt(sa);
    const double dq = 1.0 / sqrt(sb);
    const double dpq = dp * dq;
    const double hpp = a * dp * dp;
    const double hqq = b * dq * dq;
    const double2 hpq = cscale(c, dpq);
    const double2 spq = cscale(sc, dpq);

    if (hpq.x == 0.0 && hpq.y == 0.0 && spq.x == 0.0 && spq.y == 0.0) return kSkip;

    const double habs = sqrt(cnorm2(hpq));
    const double x = sqrt(cnorm2(spq));
    const double ahp = fabs(hpp), ahq = fabs(hqq);
    const double thr = crit_literal ? (fmax(ahp, ahq) * tol) * fmin(ahp, ahq)
                                    : tol * sqrt(ahp) * sqrt(ahq);
    if (!(habs >= thr || x >= tol)) return kSkip;

    // Step 1: exp(i alpha_1) = s_pq / |s_pq| (1 when s_pq = 0), S1 = diag(1+x, 1-x).
    double2 e1 = cmk(1.0, 0.0);
    if (x > 0.0) {
        const double rx = 1.0 / x;
        e1 = cscale(spq, rx);
    }
    if (!(x < 1.0)) return GHSVD_ERANK;
    const double t = sqrt((1.0 - x) * (1.0 + x));
    if (!(t > 0.0)) return GHSVD_ERANK;

    // Step 2: u + i v = conj(e1) h_pq.
    const double2 uv = cmulc(e1, hpq);
    const double u = uv.x, v = uv.y;
    const double h = hqq - hpp;

    int kind;
    double2 w11, w21, w12, w22;
    if (h == 0.0 && v == 0.0) {
        // Z = R1 D2 (Section 6.1.6).
        const double s2 = sqrt(0.5);
        const double d1 = s2 / sqrt(1.0 + x);
        const double d2 = s2 / sqrt(1.0 - x);
        w11 = cmk(d1, 0.0);
        w21 = cmk(e1.x * d1, -e1.y * d1);
        w12 = cmk(-e1.x * d2, -e1.y * d2);
        w22 = cmk(d2, 0.0);
        kind = kBig;
    } else {
        // Step 3 via (6.7) and (6.11), no trigonometric calls.
        const double sigma = (h >= 0.0) ? 1.0 : -1.0;
        const double twov = 2.0 * v;
        const double r = hypot(h, twov);
        const double cos_g = fabs(h) / r;
        const double sin_g = sigma * twov / r;
        const double num = sigma * (2.0 * u - (hpp + hqq) * x);
        const double den = t * r;
        const double rho = hypot(num, den);
        const double cos_2t = den / rho;
        const double sin_2t = num / rho;
        // (6.10)
        const double base = 1.0 + t * cos_g * cos_2t;
        const double cphi = sqrt(0.5 * (base + x * sin_2t));
        const double cpsi = sqrt(0.5 * (base - x * sin_2t));
        const double im = t * sin_g * cos_2t;
        // e^{i alpha} sin(phi) = e1 ((sin2t - x) + i im) / (2 cos psi)
        const double ka = 0.5 / cpsi;
        const double2 ea = cmul(e1, cmk((sin_2t - x) * ka, im * ka));
        // e^{-i beta} sin(psi) = conj(e1) ((sin2t + x) - i im) / (2 cos phi)
        const double kb = 0.5 / cphi;
        const double2 eb = cmul(cconj(e1), cmk((sin_2t + x) * kb, -im * kb));
        const double rt = 1.0 / t;
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

}  // namespace ghsvd
