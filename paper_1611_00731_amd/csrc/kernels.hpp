// Host-side launchers of the PUFE kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pufe.h"
#include "tables.hpp"

namespace pufe {

constexpr int kContractQ = 16;      // quadrature points per LDS stage of the contraction
constexpr int kMaxKPerLaunch = 16;  // k-points handled by one scatter launch
constexpr int kSplitQ = 32;         // quadrature points per LDS stage of the split-bf16 contraction
// Fixed device workspace of the allocation-free assembly (per GPU, held for
// the life of the process): the phase table and the K-chunk partial tiles.
constexpr size_t kScratchBytes = PUFE_NOALLOC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

struct KPoints {
    int32_t nk;
    double kap[kMaxKPerLaunch][3];
};

// Device address of the fixed workspace on `device`, which must be the
// current device; looked up once per device and kept.
hipError_t scratch_address(int device, double **ptr);

hipError_t launch_aq_geom(const KParams &kp, int64_t nel, const double *pos, int n_atoms, const double *L,
                          int max_level, double dist, int64_t *count, const int64_t *off, uint32_t *out,
                          int32_t *leaf_elem, hipStream_t st);
hipError_t launch_scan(const int64_t *in, int64_t n, int64_t *off, hipStream_t st);
hipError_t launch_qp_export(const KParams &kp, int64_t n_leaves, const uint32_t *leaves, const int32_t *leaf_elem,
                            double *xyz, double *w, hipStream_t st);
hipError_t launch_elem_qp_offset(const KParams &kp, int64_t nel, const int64_t *leaf_off, int64_t *qp_off,
                                 hipStream_t st);
hipError_t init_contract_attributes();
hipError_t init_split_attributes();
size_t contract_lds_bytes(int q, int rows, int nfun, int nimg, int nleaf, int n3);
bool contract_q_supported(int q);
hipError_t launch_contract_f64(int q, int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items,
                               const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                               const uint32_t *leaves, const double *V, double *partial, size_t lds,
                               hipStream_t st);
// Wide contraction (8-wave work groups, one per CU) for the items of elements
// of more than kWholeMaxTiles tiles.
constexpr int kWholeMaxTiles = 5;   // elements of at most 80 functions: whole-element narrow items
constexpr int kWideTiles = 6;       // tile block of the wide items
size_t contract_wide_lds_bytes(int rows, int nfun, int nimg, int nleaf, int n3);
hipError_t launch_contract_wide(int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items, const ElemDev *elems,
                                const GroupDev *groups, const double *img, const int32_t *edof, const uint32_t *leaves,
                                const double *V, double *partial, size_t lds, hipStream_t st);
hipError_t launch_contract_wide_persistent(int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items,
                                           int *counter, int grid, size_t lds, hipStream_t st);
size_t split_lds_bytes(int nlimb, int rows, int nfun, int nimg, int nleaf, int n3);
hipError_t launch_contract_split(int nlimb, int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items, const ElemDev *elems,
                                 const GroupDev *groups, const double *img, const int32_t *edof,
                                 const uint32_t *leaves, const double *V, double *partial, size_t lds,
                                 hipStream_t st);
int persistent_blocks_per_cu(size_t lds);
hipError_t launch_contract_persistent(int q, int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items,
                                      int *counter, int grid, size_t lds, hipStream_t st);
hipError_t launch_split_persistent(int nlimb, int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items, int *counter,
                                   int grid, size_t lds, hipStream_t st);
hipError_t launch_chunk_reduce(const ElemDev *elems, const int2 *list, int n, double *partial, hipStream_t st);
hipError_t launch_chunk_reduce_batch(const CtxDev *ctxs, const int4 *list, int n, hipStream_t st);
hipError_t launch_phase_table(const KPoints &kps, double2 *z, hipStream_t st);
hipError_t launch_scatter_batch(const CtxDev *ctxs, const int4 *list, int n, const double2 *z, int nk,
                                int out_dtype, hipStream_t st);
hipError_t launch_fill_zero(void *p, int64_t n, bool f32, hipStream_t st);
// zero H and S (bytes each, a multiple of 8; S may be null) and the phase table of kps, one launch
hipError_t launch_prepare_outputs(void *H, void *S, int64_t bytes, const KPoints &kps, double2 *z, hipStream_t st);
hipError_t launch_scatter(const KParams &kp, const ElemDev *elems, const int2 *list, int n, const int32_t *edof,
                          const double *partial, const double2 *z, int nk, int out_dtype, void *H, void *S,
                          int64_t nnz, hipStream_t st);
hipError_t launch_elem_matrices(const ElemDev *elems, int64_t e, const double *partial, double *He, double *Se,
                                int ld, hipStream_t st);
hipError_t launch_bsr_to_dense(int64_t nnzb, const int32_t *brow, const int32_t *bcol, const int64_t *bval_off,
                               const int64_t *dof_off, const void *src, int dtype, int64_t n, double *dense,
                               hipStream_t st);

}  // namespace pufe
