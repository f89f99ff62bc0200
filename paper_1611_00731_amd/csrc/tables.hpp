// Device-side table layouts shared by the host planner and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pufe {

constexpr int kMaxFun = 64;       // enrichment functions on one element
constexpr int kMaxGroups = 32;    // (atom, descriptor) groups on one element
constexpr int kMaxNloc = 512;     // functions on one element
constexpr int kTile = 16;         // MFMA tile edge
constexpr int kBlockTiles = 4;    // tiles per row/column block of a work item
constexpr int kMaxGauss = 12;
constexpr int kMaxLevel = 8;
constexpr int kMaxRowChunks = 64; // enriched-row chunks of one partial work item
constexpr int kMaxProjCols = 64;  // projector columns reaching one element
constexpr int kMaxPGroups = 32;   // projector-image groups reaching one element
// dynamic LDS a kernel may request: the 160 KiB of a CU minus room for the
// small static __shared__ variables some kernels also declare
constexpr size_t kMaxDynLds = 159 * 1024;

// One element: geometry index, function counts, table offsets and the BSR
// addresses of its 8x8 corner-vertex blocks.
struct ElemDev {
    int32_t nloc, nfe, nfun, ngrp;
    int32_t grp_off, edof_off;
    int32_t ijk[3];
    int32_t color;
    int32_t shifts;      // lattice shift bits of corner c at bits 3c..3c+2 (bit d = direction d)
    int32_t nchunk;      // K-chunks of the contraction
    int64_t leaf_off, leaf_end;
    int64_t part_base;   // first partial tile-pair slot
    int64_t blk[64];     // value offset of BSR block (vertex of corner ca, vertex of corner cb) at ca*8+cb
    int32_t bw[8];       // width of the block column of corner c (b_w of its vertex)
    int32_t pg_off, npg; // projector-image groups reaching the element
    int32_t ncol;        // projector columns (sum of 2l+1 over the groups)
    int32_t pf_nchunk;   // K-chunks of its projector coefficients (0: none)
    int64_t pf_base;     // first double of its projector-coefficient slots, F[chunk][col][npad]
};

// Projector descriptor of one atom image that reaches an element: the 2l+1
// columns col0 .. col0 + 2l of the element's projector coefficients, the
// projector functions J0 .. J0 + 2l, the image centre and its lattice shift.
struct PGroupDev {
    double c[3];
    double a, rc;
    int32_t l, col0, J0, n[3];
};

// A nonlocal work item: one element, one range of its octree leaves, one row
// block of its local functions (tiles R0 .. R0 + nR - 1).
struct NlItemDev {
    int32_t elem, chunk, R0, nR;
    int64_t leaf_b, leaf_e;
};

// (atom, descriptor) group: 2l+1 functions with one radial part and the list
// of lattice images whose cutoff sphere reaches the element.  A tabulated
// radial (nspl > 0 intervals of width rc / nspl, a = nspl / rc) is the cubic
// on interval j = floor(a r) with coefficients spl[spl_off + 4 j + 0..3] in
// powers of tau = a r - j.
struct GroupDev {
    int32_t atom, desc, l, fbase, img_off, nimg, nspl, spl_off;
    double a, rc;   // a: Gaussian exponent (analytic) or intervals per bohr (tabulated)
};

// Serendipity elements (fe_order 3): the k-th (k = 0..3) corner whose bit d
// is clear, where edge 4 d + k along direction d starts.
static inline __host__ __device__ int serendipity_edge_corner(int d, int k) {
    const int low = k & ((1 << d) - 1);
    return low | ((k >> d) << (d + 1));
}

// Enriched local function: corner | element-function << 3 | vertex slot << 11
static inline __host__ __device__ int32_t edof_pack(int corner, int f, int slot) {
    return corner | (f << 3) | (slot << 11);
}

// A contraction work item: one element, one row block and one column block of
// 16x16 tiles, one range of octree leaves (a K-chunk).
struct ItemDev {
    int32_t elem, I0, nI, J0, nJ, chunk;
    int64_t leaf_b, leaf_e;
    int32_t ctx;         // problem of a batched launch (0 otherwise)
};

// Per-launch constants of the mesh and the rule.
struct KParams {
    double E[9];      // row d: a_d / n_d (element edge vector)
    double Jt[9];     // grad_x[c] = sum_d Jt[3c+d] dphi/dxi_d
    double jac;       // det of the reference-to-element map
    double gx[kMaxGauss], gw[kMaxGauss];   // base rule (n points)
    double rx[kMaxGauss], rw[kMaxGauss];   // reference rule of the error mode (nref points)
    int32_t n, n3, p, nfe, nfs, nref;
    int32_t mesh[3];
    const double *spl;   // coefficients of the tabulated radials (device)
    // Bloch-periodic enrichment: the weight of every image entry at the
    // k-point of the launch, cos or sin(2 pi kappa.n) (null: periodic, all 1)
    const double *wimg;
};

// Tables and buffers of one problem, for launches that cover several problems
// (one per lattice constant of a sweep).
struct CtxDev {
    KParams kp;
    const ElemDev *elems;
    const GroupDev *groups;
    const double *img;
    const int32_t *edof;
    const uint32_t *leaves;
    const double *V;
    double *partial;
    void *H, *S;
    int64_t nnz;
};

// Octree cell of the error-driven rule builder: element, leaf code, and the
// bit mask of the element's enrichment functions still tested on it.
struct CellDev {
    uint64_t mask;
    int32_t elem;
    uint32_t code;
    int32_t open;   // 1 while the cell may still split
    int32_t pad;
};

// Leaf code: level in bits 27..30, cell coordinates in 9-bit fields.
static inline __host__ __device__ uint32_t leaf_pack(int lev, int c1, int c2, int c3) {
    return (uint32_t)c1 | ((uint32_t)c2 << 9) | ((uint32_t)c3 << 18) | ((uint32_t)lev << 27);
}

}  // namespace pufe
