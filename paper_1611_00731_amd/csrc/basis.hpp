// Device building blocks of the enriched PUFE basis (eq. pufebasis):
// 1D Lagrange factors of the classical FE functions, trilinear PU factors,
// real solid harmonics and the cut-off Gaussian radial part of the enrichment.
#pragma once
#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace pufe {

// r^l Y_lm normalisations (orthonormal real harmonics, no Condon-Shortley phase)
constexpr double Y0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double Y1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double Y2A = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double Y2B = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double Y2C = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double Y3A = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double Y3B = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double Y3C = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double Y3D = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double Y3E = 1.445305721320277;    // sqrt(105/pi)/4

// Solid harmonics S_m = r^l Y_lm(r_hat) for m = -l..l (index m + l) and their
// gradients g[3 * (m + l) + c] at r = (x, y, z).
__device__ __forceinline__ void solid_harmonics(int l, double x, double y, double z, double *S, double *g) {
    if (l == 0) {
        S[0] = Y0;
        g[0] = g[1] = g[2] = 0.0;
    } else if (l == 1) {
        S[0] = Y1 * y; g[0] = 0.0; g[1] = Y1;  g[2] = 0.0;
        S[1] = Y1 * z; g[3] = 0.0; g[4] = 0.0; g[5] = Y1;
        S[2] = Y1 * x; g[6] = Y1;  g[7] = 0.0; g[8] = 0.0;
    } else if (l == 2) {
        double xx = x * x, yy = y * y, zz = z * z;
        S[0] = Y2A * x * y;               g[0] = Y2A * y;        g[1] = Y2A * x;        g[2] = 0.0;
        S[1] = Y2A * y * z;               g[3] = 0.0;            g[4] = Y2A * z;        g[5] = Y2A * y;
        S[2] = Y2B * (2.0 * zz - xx - yy); g[6] = -2.0 * Y2B * x; g[7] = -2.0 * Y2B * y; g[8] = 4.0 * Y2B * z;
        S[3] = Y2A * x * z;               g[9] = Y2A * z;        g[10] = 0.0;           g[11] = Y2A * x;
        S[4] = Y2C * (xx - yy);           g[12] = 2.0 * Y2C * x; g[13] = -2.0 * Y2C * y; g[14] = 0.0;
    } else {
        double xx = x * x, yy = y * y, zz = z * z;
        double t = 4.0 * zz - xx - yy;
        S[0] = Y3A * y * (3.0 * xx - yy);
        g[0] = 6.0 * Y3A * x * y; g[1] = 3.0 * Y3A * (xx - yy); g[2] = 0.0;
        S[1] = Y3B * x * y * z;
        g[3] = Y3B * y * z; g[4] = Y3B * x * z; g[5] = Y3B * x * y;
        S[2] = Y3C * y * t;
        g[6] = -2.0 * Y3C * x * y; g[7] = Y3C * (4.0 * zz - xx - 3.0 * yy); g[8] = 8.0 * Y3C * y * z;
        S[3] = Y3D * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
        g[9] = -6.0 * Y3D * x * z; g[10] = -6.0 * Y3D * y * z; g[11] = 3.0 * Y3D * (2.0 * zz - xx - yy);
        S[4] = Y3C * x * t;
        g[12] = Y3C * (4.0 * zz - 3.0 * xx - yy); g[13] = -2.0 * Y3C * x * y; g[14] = 8.0 * Y3C * x * z;
        S[5] = Y3E * z * (xx - yy);
        g[15] = 2.0 * Y3E * x * z; g[16] = -2.0 * Y3E * y * z; g[17] = Y3E * (xx - yy);
        S[6] = Y3A * x * (xx - 3.0 * yy);
        g[18] = 3.0 * Y3A * (xx - yy); g[19] = -6.0 * Y3A * x * y; g[20] = 0.0;
    }
}

// Hessians of the solid harmonics, 6 symmetric components per m
// (xx, yy, zz, xy, xz, yz) at h[6 * (m + l) + c].
__device__ __forceinline__ void solid_harmonics_hess(int l, double x, double y, double z, double *h) {
    const int nm = 2 * l + 1;
    for (int k = 0; k < 6 * nm; ++k) h[k] = 0.0;
    if (l == 2) {
        h[0 * 6 + 3] = Y2A;                                   // xy
        h[1 * 6 + 5] = Y2A;                                   // yz
        h[2 * 6 + 0] = -2.0 * Y2B; h[2 * 6 + 1] = -2.0 * Y2B; h[2 * 6 + 2] = 4.0 * Y2B;
        h[3 * 6 + 4] = Y2A;                                   // xz
        h[4 * 6 + 0] = 2.0 * Y2C; h[4 * 6 + 1] = -2.0 * Y2C;
    } else if (l == 3) {
        double *m;
        m = h + 0 * 6; m[0] = 6.0 * Y3A * y; m[1] = -6.0 * Y3A * y; m[3] = 6.0 * Y3A * x;
        m = h + 1 * 6; m[3] = Y3B * z; m[4] = Y3B * y; m[5] = Y3B * x;
        m = h + 2 * 6; m[0] = -2.0 * Y3C * y; m[1] = -6.0 * Y3C * y; m[2] = 8.0 * Y3C * y;
                       m[3] = -2.0 * Y3C * x; m[5] = 8.0 * Y3C * z;
        m = h + 3 * 6; m[0] = -6.0 * Y3D * z; m[1] = -6.0 * Y3D * z; m[2] = 12.0 * Y3D * z;
                       m[4] = -6.0 * Y3D * x; m[5] = -6.0 * Y3D * y;
        m = h + 4 * 6; m[0] = -6.0 * Y3C * x; m[1] = -2.0 * Y3C * x; m[2] = 8.0 * Y3C * x;
                       m[3] = -2.0 * Y3C * y; m[4] = 8.0 * Y3C * z;
        m = h + 5 * 6; m[0] = 2.0 * Y3E * z; m[1] = -2.0 * Y3E * z; m[4] = 2.0 * Y3E * x; m[5] = -2.0 * Y3E * y;
        m = h + 6 * 6; m[0] = 6.0 * Y3A * x; m[1] = -6.0 * Y3A * x; m[3] = -6.0 * Y3A * y;
    }
}

// 1D Lagrange factors of order p (1 or 2) on the nodes -1, (0,) 1 of the
// reference interval: values L[0..p] and derivatives D[0..p] at t.
__device__ __forceinline__ void lagrange_1d(int p, double t, double *L, double *D) {
    if (p == 1) {
        L[0] = 0.5 * (1.0 - t); L[1] = 0.5 * (1.0 + t);
        D[0] = -0.5;            D[1] = 0.5;
    } else {
        L[0] = 0.5 * t * (t - 1.0); L[1] = 1.0 - t * t; L[2] = 0.5 * t * (t + 1.0);
        D[0] = t - 0.5;             D[1] = -2.0 * t;    D[2] = t + 0.5;
    }
}

// 32-node cubic serendipity hexahedron (fe_order 3).  Local FE function a:
// a < 8 the corner a (coordinates -1 + 2 bit_d(a)); a = 8 + 2 e + t the node
// at -1/3 (t = 0) or +1/3 (t = 1) of edge e = 4 d + k along direction d,
// starting at the k-th corner whose bit d is clear.  With the node at
// (n_0, n_1, n_2):
//   corner:          prod_d (1 + n_d xi_d) (9 |xi|^2 - 19) / 64,
//   edge along d:  9 (1 - xi_d^2)(1 + 9 n_d xi_d) prod_{k != d} (1 + n_k xi_k) / 64.
__device__ __forceinline__ void serendipity_fn(int a, const double *xi, double *val, double *dxi) {
    if (a < 8) {
        double f[3], n[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            n[d] = ((a >> d) & 1) ? 1.0 : -1.0;
            f[d] = 1.0 + n[d] * xi[d];
        }
        const double r = 9.0 * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) - 19.0, f3 = f[0] * f[1] * f[2];
        *val = f3 * r * (1.0 / 64.0);
        dxi[0] = (n[0] * f[1] * f[2] * r + 18.0 * f3 * xi[0]) * (1.0 / 64.0);
        dxi[1] = (n[1] * f[0] * f[2] * r + 18.0 * f3 * xi[1]) * (1.0 / 64.0);
        dxi[2] = (n[2] * f[0] * f[1] * r + 18.0 * f3 * xi[2]) * (1.0 / 64.0);
        return;
    }
    const int e = (a - 8) >> 1, t = (a - 8) & 1, d = e >> 2, c = serendipity_edge_corner(d, e & 3);
    double f[3], df[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k == d) {
            const double nd = t ? (1.0 / 3.0) : (-1.0 / 3.0), x = xi[k], g = 1.0 + 9.0 * nd * x;
            f[k] = (1.0 - x * x) * g;
            df[k] = -2.0 * x * g + (1.0 - x * x) * 9.0 * nd;
        } else {
            const double nk = ((c >> k) & 1) ? 1.0 : -1.0;
            f[k] = 1.0 + nk * xi[k];
            df[k] = nk;
        }
    }
    constexpr double s = 9.0 / 64.0;
    *val = s * f[0] * f[1] * f[2];
    dxi[0] = s * df[0] * f[1] * f[2];
    dxi[1] = s * f[0] * df[1] * f[2];
    dxi[2] = s * f[0] * f[1] * df[2];
}

}  // namespace pufe
