// Enrichment functions of one (atom, descriptor) group at one point, shared
// by the FP64 and split-precision contraction kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "basis.hpp"
#include "tables.hpp"

namespace pufe {

// Enrichment functions of one (atom, descriptor) group at one point x:
// Psi_m = sum over images of g(s) S_m(r), grad Psi_m = 2 g'(s) r S_m + g grad S_m,
// g(s) = exp(-a s) (1 - s/rc^2)^3, r = x - image centre, s = |r|^2 < rc^2.
template <int L>
__device__ __forceinline__ void group_eval_point(const GroupDev &G, const double *__restrict__ img, const double *x,
                                                 double *psi, double *gp) {
    constexpr int NM = 2 * L + 1;
#pragma unroll
    for (int m = 0; m < NM; ++m) psi[m] = gp[3 * m] = gp[3 * m + 1] = gp[3 * m + 2] = 0.0;
    const double rc2 = G.rc * G.rc, inv_rc2 = 1.0 / rc2;
    const double *c0 = img + 3 * G.img_off;
    for (int k = 0; k < G.nimg; ++k) {
        const double rx = x[0] - c0[3 * k], ry = x[1] - c0[3 * k + 1], rz = x[2] - c0[3 * k + 2];
        const double s = rx * rx + ry * ry + rz * rz;
        if (s >= rc2) continue;
        const double ex = exp(-G.a * s), c = 1.0 - s * inv_rc2, c2 = c * c;
        const double g0 = ex * c2 * c;
        const double g1 = -ex * c2 * (G.a * c + 3.0 * inv_rc2);
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

// Written to o[m * MS + c * CS], c = 0 value, 1..3 gradient.
template <int L, int MS, int CS>
__device__ __forceinline__ void group_eval(const GroupDev &G, const double *__restrict__ img, const double *x,
                                           double *o) {
    constexpr int NM = 2 * L + 1;
    double psi[NM], gp[3 * NM];
    group_eval_point<L>(G, img, x, psi, gp);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        double *om = o + (size_t)m * MS;
        om[0] = psi[m];
        om[CS] = gp[3 * m];
        om[2 * CS] = gp[3 * m + 1];
        om[3 * CS] = gp[3 * m + 2];
    }
}

}  // namespace pufe
