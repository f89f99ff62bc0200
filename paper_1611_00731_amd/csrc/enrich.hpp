// Enrichment functions of one (atom, descriptor) group at one point, shared
// by the FP64 and split-precision contraction kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "basis.hpp"
#include "tables.hpp"

namespace pufe {

// Tabulated radial u at r = sqrt(s) (0 <= r < rc) written as a function of s:
// g = u, g1 = dg/ds = u'/(2r), and, when G2, g2 = d2g/ds2 = (u'' - u'/r)/(4 s).
// Piece j in tau = a r - j: u = c0 + c1 tau + c2 tau^2 + c3 tau^3, u' = a du/dtau,
// u'' = a^2 d2u/dtau2.  On the first piece the clamped slope makes c1 zero,
// so u'/r = a^2 (2 c2 + 3 c3 tau) there without a division (finite at the
// nucleus); g2 then behaves like 1/r and only enters multiplied by r r^T, so
// it is taken as 0 at r = 0.
template <bool G2>
__device__ __forceinline__ void spline_radial(const GroupDev &G, const double *__restrict__ spl, double s, double &g0,
                                              double &g1, double &g2) {
    const double r = sqrt(s), ar = G.a * r;
    const int j = min((int)ar, G.nspl - 1);
    const double *c = spl + G.spl_off + 4 * j;
    const double t = ar - j, a2 = G.a * G.a;
    g0 = c[0] + t * (c[1] + t * (c[2] + t * c[3]));
    const double u1r = j == 0 ? a2 * (2.0 * c[2] + 3.0 * c[3] * t) : G.a * (c[1] + t * (2.0 * c[2] + 3.0 * c[3] * t)) / r;
    g1 = 0.5 * u1r;
    if (G2) {
        const double u2 = a2 * (2.0 * c[2] + 6.0 * c[3] * t);
        g2 = s > 0.0 ? (u2 - u1r) / (4.0 * s) : 0.0;
    }
}

// Enrichment functions of one (atom, descriptor) group at one point x:
// Psi_m = sum over images of g(s) S_m(r), grad Psi_m = 2 g'(s) r S_m + g grad S_m,
// r = x - image centre, s = |r|^2 < rc^2; g(s) = exp(-a s) (1 - s/rc^2)^3 for
// the analytic radial, the tabulated spline otherwise.  TAB = false compiles
// the analytic radial only (kernels of problems without tabulated radials).
template <int L, bool TAB = true>
__device__ __forceinline__ void group_eval_point(const GroupDev &G, const double *__restrict__ img,
                                                 const double *__restrict__ spl, const double *x, double *psi,
                                                 double *gp) {
    constexpr int NM = 2 * L + 1;
#pragma unroll
    for (int m = 0; m < NM; ++m) psi[m] = gp[3 * m] = gp[3 * m + 1] = gp[3 * m + 2] = 0.0;
    const double rc2 = G.rc * G.rc, inv_rc2 = 1.0 / rc2;
    const double *c0 = img + 3 * G.img_off;
    for (int k = 0; k < G.nimg; ++k) {
        const double rx = x[0] - c0[3 * k], ry = x[1] - c0[3 * k + 1], rz = x[2] - c0[3 * k + 2];
        const double s = rx * rx + ry * ry + rz * rz;
        if (s >= rc2) continue;
        double g0, g1;
        if (TAB && G.nspl > 0) {
            double unused;
            spline_radial<false>(G, spl, s, g0, g1, unused);
        } else {
            const double ex = exp(-G.a * s), c = 1.0 - s * inv_rc2, c2 = c * c;
            g0 = ex * c2 * c;
            g1 = -ex * c2 * (G.a * c + 3.0 * inv_rc2);
        }
        double S[7], dS[21];
        solid_harmonics(L, rx, ry, rz, S, dS);
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            psi[m] += g0 * S[m];
            gp[3 * m] += 2.0 * g1 * rx * S[m] + g0 * dS[3 * m];
            gp[3 * m + 1] += 2.0 * g1 * ry * S[m] + g0 * dS[3 * m + 1];
            gp[3 * m + 2] += 2.0 * g1 * rz * S[m] + g0 * dS[3 * m + 2];
        }
    }
}

// Written to o[m * MS + c * CS], c = 0 value, 1..3 gradient.  The sums over
// images accumulate in place (the first image writes, later ones add), so no
// per-function accumulators stay live in registers.  With TAB, a non-null
// wimg weights image k by wimg[G.img_off + k] (eq. Psi with
// f(R) = exp(i k.R): the real and the imaginary part of a Bloch-periodic
// enrichment function are two groups with cos and sin weights).
template <int L, int MS, int CS, bool TAB = true>
__device__ __forceinline__ void group_eval(const GroupDev &G, const double *__restrict__ img,
                                           const double *__restrict__ spl, const double *__restrict__ wimg,
                                           const double *x, double *o) {
    constexpr int NM = 2 * L + 1;
    const double rc2 = G.rc * G.rc, inv_rc2 = 1.0 / rc2;
    const double *c0 = img + 3 * G.img_off;
    bool first = true;
    for (int k = 0; k < G.nimg; ++k) {
        const double rx = x[0] - c0[3 * k], ry = x[1] - c0[3 * k + 1], rz = x[2] - c0[3 * k + 2];
        const double s = rx * rx + ry * ry + rz * rz;
        if (s >= rc2) continue;
        double g0, g1;
        if (TAB && G.nspl > 0) {
            double unused;
            spline_radial<false>(G, spl, s, g0, g1, unused);
        } else {
            const double ex = exp(-G.a * s), c = 1.0 - s * inv_rc2, c2 = c * c;
            g0 = ex * c2 * c;
            g1 = -ex * c2 * (G.a * c + 3.0 * inv_rc2);
        }
        if (TAB && wimg) {
            const double wk = wimg[G.img_off + k];
            g0 *= wk;
            g1 *= wk;
        }
        double S[7], dS[21];
        solid_harmonics(L, rx, ry, rz, S, dS);
        const double tx = 2.0 * g1 * rx, ty = 2.0 * g1 * ry, tz = 2.0 * g1 * rz;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double *om = o + (size_t)m * MS;
            const double v0 = g0 * S[m], v1 = tx * S[m] + g0 * dS[3 * m], v2 = ty * S[m] + g0 * dS[3 * m + 1],
                         v3 = tz * S[m] + g0 * dS[3 * m + 2];
            if (first) {
                om[0] = v0;
                om[CS] = v1;
                om[2 * CS] = v2;
                om[3 * CS] = v3;
            } else {
                om[0] += v0;
                om[CS] += v1;
                om[2 * CS] += v2;
                om[3 * CS] += v3;
            }
        }
        first = false;
    }
    if (first)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double *om = o + (size_t)m * MS;
            om[0] = om[CS] = om[2 * CS] = om[3 * CS] = 0.0;
        }
}

}  // namespace pufe
