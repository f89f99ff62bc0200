// Host-side launchers of the adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace pufe {

constexpr int kBackwardQ = 16;         // quadrature points per LDS stage of the adjoint
constexpr int kBackwardMaxNloc = 80;   // largest element the block-resident adjoint kernel holds (5 row tiles)
constexpr int kBwBlock = 64;           // functions per row/column block of the wide adjoint kernel
constexpr int kBackwardWideMaxEnr = 256;   // enriched functions of one element the wide kernel holds

hipError_t init_backward_attributes();
size_t backward_lds_bytes(int npad, int nenr, int nfun, int nimg);
hipError_t launch_gather_adjoint(const KParams &kp, int64_t nel, const ElemDev *elems, const int32_t *edof,
                                 const int64_t *pt_off, const double *P, const double *kpt, double *Pt,
                                 hipStream_t st);
// nl = 0: FP64 MFMA form; nl = 2 or 3: split-precision form (bf16 limbs per operand)
hipError_t launch_backward(const KParams &kp, bool qmode, int nl, int n_items, const ItemDev *items,
                           const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                           const uint32_t *leaves, const double *V, const int64_t *pt_off, const double *Pt,
                           double *dLdV, double *fpart, int max_ngrp, size_t lds, hipStream_t st);
// Elements of more than kBackwardMaxNloc functions, FP64 (row x column
// blocks of Ps streamed through LDS every stage).
size_t backward_wide_lds_bytes(int nfun, int nimg);
hipError_t launch_backward_wide(const KParams &kp, bool qmode, int n_items, const ItemDev *items,
                                const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                                const uint32_t *leaves, const double *V, const int64_t *pt_off, const double *Pt,
                                double *dLdV, double *fpart, int max_ngrp, size_t lds, hipStream_t st);
hipError_t launch_force_reduce(int n_atoms, const int64_t *atom_ptr, const int64_t *atom_slots, const double *fP,
                               const double *fQ, double *dLdR, hipStream_t st);

}  // namespace pufe
