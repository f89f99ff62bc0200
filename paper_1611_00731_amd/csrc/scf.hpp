// Launchers of the self-consistent field kernels (scf.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace pufe {

// Load vector of the classical FE space, b[v * nfs + s] = sum_q w_q phi f_q:
// per-element sums into be (nel x 32), then a gather per DOF over its
// (element, local function) pairs.
hipError_t launch_fe_load(const KParams &kp, const ElemDev *elems, int64_t nel, const uint32_t *leaves,
                          const double *f, double *be, int64_t nv, int nfs, const int64_t *dof_off,
                          const int64_t *dof_el_off, const int2 *dof_el, double *b, hipStream_t st);
// out_q = sum_i u_i phi_i(x_q) over the classical FE functions.
hipError_t launch_fe_eval(const KParams &kp, const ElemDev *elems, const int32_t *edof, const uint32_t *leaves,
                          const int32_t *leaf_elem, int64_t n_qp, const double *u, double *out, hipStream_t st);
// The nfs x nfs classical FE corner of every BSR block of A, times scale.
hipError_t launch_fe_blocks(int64_t nnzb, int nfs, const int32_t *bcol, const int64_t *bval_off,
                            const int64_t *dof_off, const double *A, double scale, double *K, hipStream_t st);
hipError_t launch_fe_spmv(int64_t nv, int nfs, const int64_t *brow_ptr, const int32_t *bcol, const double *K,
                          const double *x, double *y, hipStream_t st);
// *out = a . b in a fixed order; part holds dot_partial_slots() doubles.
hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, hipStream_t st);
int dot_partial_slots();
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st);
hipError_t launch_scaled_diff(int64_t n, double a, const double *x, double c, const double *z, double *y,
                              hipStream_t st);
hipError_t launch_lda_xc(int64_t n, const double *rho, double *vxc, double *exc, hipStream_t st);

}  // namespace pufe
