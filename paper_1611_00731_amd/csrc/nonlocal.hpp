// Host launchers of the separable nonlocal term (nonlocal.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "tables.hpp"

namespace pufe {

size_t nl_lds_bytes(int npad, int ncol, int nfun, int nimg, int nleaf, int n3);
hipError_t init_nonlocal_attributes();
hipError_t launch_nl_f(int lmax, const KParams &kp, int n_items, const NlItemDev *items, const ElemDev *elems,
                       const GroupDev *groups, const double *img, const int32_t *edof, const uint32_t *leaves,
                       const PGroupDev *pgroups, double *Fp, size_t lds, hipStream_t st);
hipError_t launch_nl_reduce(const ElemDev *elems, const int32_t *nl_elems, int n, double *Fp, hipStream_t st);
// bpart: the partner table of the Bloch-periodic enrichment's rows (null for
// the periodic form)
hipError_t launch_nl_gather(const KParams &kp, const ElemDev *elems, const PGroupDev *pgroups, const int32_t *edof,
                            const int32_t *bpart, const int64_t *dof_el_off, const int2 *dof_el, const double *Fp,
                            const KPoints &kps, int n_pfun, int64_t n_dof, double2 *f, hipStream_t st);
hipError_t launch_nl_update(int n_blocks, const int32_t *nl_blocks, const int32_t *brow, const int32_t *bcol,
                            const int64_t *bval_off, const int64_t *dof_off, const double2 *f, const double *pfun_h,
                            int n_pfun, int64_t n_dof, int nk, int out_dtype, void *H, int64_t nnz, hipStream_t st);

}  // namespace pufe
