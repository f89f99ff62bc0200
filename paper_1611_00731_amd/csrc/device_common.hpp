// Device helpers shared by the forward and adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace pufe {

// Reference point and weight of Gauss point j of a leaf.
__device__ __forceinline__ void leaf_point(const KParams &kp, uint32_t code, int j, double *xi, double *w) {
    int lev = (int)(code >> 27);
    int c[3] = {(int)(code & 511u), (int)((code >> 9) & 511u), (int)((code >> 18) & 511u)};
    int k[3] = {j % kp.n, (j / kp.n) % kp.n, j / (kp.n * kp.n)};
    double h = 1.0 / (double)(1 << lev);
    double wt = h * h * h * kp.jac;
    for (int d = 0; d < 3; ++d) {
        xi[d] = -1.0 + (2.0 * c[d] + 1.0 + kp.gx[k[d]]) * h;
        wt *= kp.gw[k[d]];
    }
    *w = wt;
}

// corner and vertex slot of local function a
__device__ __forceinline__ void local_slot(const ElemDev &el, const int32_t *edof, int p, int a, int *corner,
                                           int *slot) {
    if (a < el.nfe) {
        if (p == 1) {
            *corner = a;
            *slot = 0;
        } else if (p == 3) {   // serendipity: corners, then two nodes per edge (slots 1 + 2 d + t)
            if (a < 8) {
                *corner = a;
                *slot = 0;
            } else {
                const int e = (a - 8) >> 1, d = e >> 2;
                *corner = serendipity_edge_corner(d, e & 3);
                *slot = 1 + 2 * d + ((a - 8) & 1);
            }
        } else {
            int d0 = a % 3, d1 = (a / 3) % 3, d2 = a / 9;
            *corner = (d0 == 2) | ((d1 == 2) << 1) | ((d2 == 2) << 2);
            *slot = (d0 == 1) | ((d1 == 1) << 1) | ((d2 == 1) << 2);
        }
    } else {
        int pk = edof[el.edof_off + (a - el.nfe)];
        *corner = pk & 7;
        *slot = pk >> 11;
    }
}

}  // namespace pufe
