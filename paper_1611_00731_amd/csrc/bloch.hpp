// Launchers of the Bloch-periodic enrichment kernels (bloch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace pufe {

// Image weights of one k-point: w[i] = cos or sin(2 pi kappa.n_i) by the
// kind of entry i (img_nk: 4 ints per entry, the lattice shift and the kind).
hipError_t launch_image_weights(const int32_t *img_nk, int64_t n, const double kap[3], double *w, hipStream_t st);

// Complex scatter of one colour at one k-point: list[n] (element, upper tile
// pair), bpart the partner table of the enriched entries, z the 27 phase
// factors of the k-point, H and S that k-point's output arrays.
hipError_t launch_scatter_bloch(const KParams &kp, const ElemDev *elems, const int2 *list, int n,
                                const int32_t *edof, const int32_t *bpart, const double *partial, const double2 *z,
                                int out_dtype, void *H, void *S, hipStream_t st);

}  // namespace pufe
