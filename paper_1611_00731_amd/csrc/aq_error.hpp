// Launchers of the error-driven rule builder.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.hpp"

namespace pufe {

hipError_t launch_aq_error_init(int64_t nel, const ElemDev *elems, CellDev *cells, hipStream_t st);
hipError_t launch_aq_error_test(const KParams &kp, const ElemDev *elems, const GroupDev *groups, const double *img,
                                const CellDev *cells, int64_t n, int max_level, double tol, int64_t *count,
                                uint64_t *newmask, hipStream_t st);
hipError_t launch_aq_error_expand(int64_t n, const CellDev *cells, const int64_t *off, const uint64_t *newmask,
                                  CellDev *next, hipStream_t st);
hipError_t launch_aq_error_finish(int64_t n, const CellDev *cells, uint32_t *leaves, int32_t *leaf_elem,
                                  int64_t *count, hipStream_t st);

}  // namespace pufe
