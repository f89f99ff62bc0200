// HIP kernels of the PUFE assembly for gfx950 (MI355X).
//
//   aq_*            adaptive quadrature: octree leaves per element (section
//                   "Adaptive quadrature"), geometric refinement mode
//   contract_f64    fused basis evaluation + FP64 MFMA contraction of the
//                   element matrices H_e = B W_H B^T, S_e = B W B^T (eq. disceig3d)
//   scatter         Bloch phases + atomic-free coloured scatter into the
//                   block-sparse H and S (one launch per element colour)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "basis.hpp"
#include "device_common.hpp"
#include "enrich.hpp"
#include "kernels.hpp"
#include "stage.hpp"
#include "tables.hpp"

namespace pufe {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- quadrature

// Closest distance^2 from the axis-aligned box [lo, hi] to any lattice image
// of the atoms of an orthorhombic cell (side lengths L).
__device__ double box_nucleus_dist2(const double *lo, const double *hi, const double *L,
                                    const double *pos, int n_atoms) {
    double best = 1e300;
    for (int A = 0; A < n_atoms; ++A) {
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            double mid = 0.5 * (lo[d] + hi[d]), half = 0.5 * (hi[d] - lo[d]);
            double t = pos[3 * A + d];
            double y = t - L[d] * rint((t - mid) / L[d]);   // image nearest to the centre
            double dd = fabs(y - mid) - half;
            if (dd > 0.0) d2 += dd * dd;
        }
        best = fmin(best, d2);
    }
    return best;
}

// One thread per element walks its octree depth first (children c = c1 +
// 2 c2 + 4 c3 in order); a cell splits while its level is below max_level
// and it lies within `dist` of a nucleus image.  With out == nullptr only the
// leaves are counted.
__global__ void aq_geom_kernel(const KParams kp, int64_t nel, const double *__restrict__ pos, int n_atoms,
                               double L0, double L1, double L2, int max_level, double dist2,
                               int64_t *__restrict__ count, const int64_t *__restrict__ off,
                               uint32_t *__restrict__ out, int32_t *__restrict__ leaf_elem) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nel) return;
    const double L[3] = {L0, L1, L2};
    int i[3] = {(int)(e % kp.mesh[0]), (int)((e / kp.mesh[0]) % kp.mesh[1]),
                (int)(e / ((int64_t)kp.mesh[0] * kp.mesh[1]))};
    double h[3] = {L0 / kp.mesh[0], L1 / kp.mesh[1], L2 / kp.mesh[2]};
    uint32_t stack[8 * kMaxLevel + 2];
    int sp = 0;
    stack[sp++] = leaf_pack(0, 0, 0, 0);
    int64_t n = 0, base = out ? off[e] : 0;
    while (sp > 0) {
        uint32_t code = stack[--sp];
        int lev = (int)(code >> 27);
        int c[3] = {(int)(code & 511u), (int)((code >> 9) & 511u), (int)((code >> 18) & 511u)};
        bool split = false;
        if (lev < max_level) {
            double lo[3], hi[3], s = 1.0 / (double)(1 << lev);
            for (int d = 0; d < 3; ++d) {
                lo[d] = (i[d] + c[d] * s) * h[d];
                hi[d] = (i[d] + (c[d] + 1) * s) * h[d];
            }
            split = box_nucleus_dist2(lo, hi, L, pos, n_atoms) <= dist2;
        }
        if (split) {
            for (int ch = 7; ch >= 0; --ch)
                stack[sp++] = leaf_pack(lev + 1, 2 * c[0] + (ch & 1), 2 * c[1] + ((ch >> 1) & 1),
                                        2 * c[2] + ((ch >> 2) & 1));
        } else {
            if (out) {
                out[base + n] = code;
                leaf_elem[base + n] = (int32_t)e;
            }
            ++n;
        }
    }
    if (!out) count[e] = n;
}

// Exclusive scan of n int64 values into off[0..n] by one workgroup of 1024.
__global__ __launch_bounds__(1024) void scan_kernel(const int64_t *__restrict__ in, int64_t n,
                                                    int64_t *__restrict__ off) {
    __shared__ int64_t part[1024];
    int t = threadIdx.x;
    int64_t per = (n + 1023) / 1024;
    int64_t b = t * per, e = b + per < n ? b + per : n;
    int64_t s = 0;
    for (int64_t k = b; k < e; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int stride = 1; stride < 1024; stride <<= 1) {
        int64_t v = t >= stride ? part[t - stride] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t k = b; k < e; ++k) {
        off[k] = run;
        run += in[k];
    }
    if (t == 1023) off[n] = part[1023];
}

__global__ void qp_export_kernel(const KParams kp, int64_t n_leaves, const uint32_t *__restrict__ leaves,
                                 const int32_t *__restrict__ leaf_elem, double *__restrict__ xyz,
                                 double *__restrict__ w) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_leaves * kp.n3) return;
    int64_t lf = q / kp.n3;
    int j = (int)(q % kp.n3);
    int64_t e = leaf_elem[lf];
    int i[3] = {(int)(e % kp.mesh[0]), (int)((e / kp.mesh[0]) % kp.mesh[1]),
                (int)(e / ((int64_t)kp.mesh[0] * kp.mesh[1]))};
    double xi[3], wt;
    leaf_point(kp, leaves[lf], j, xi, &wt);
    if (w) w[q] = wt;
    if (xyz)
        for (int c = 0; c < 3; ++c) {
            double x = 0.0;
            for (int d = 0; d < 3; ++d) x += (i[d] + 0.5 * (xi[d] + 1.0)) * kp.E[3 * d + c];
            xyz[3 * q + c] = x;
        }
}

__global__ void elem_qp_offset_kernel(const KParams kp, int64_t nel, const int64_t *__restrict__ leaf_off,
                                      int64_t *__restrict__ qp_off) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e <= nel) qp_off[e] = leaf_off[e] * kp.n3;
}

// ---------------------------------------------------------- contraction
//
// One work group of 4 waves per work item; each stage of Q points runs three
// phases separated by barriers:
//   1. enrichment functions at the stage points (group, point pairs), while
//      the last Q threads build the per-point geometry;
//   2. the weighted rows of the item's local functions;
//   3. FP64 MFMAs over the item's 16x16 tile pairs, round-robin over waves.
// FP64 MFMAs and FP64 VALU instructions do not co-issue on one SIMD, so the
// phases are kept lean and the LDS footprint small enough for two work
// groups per CU, whose phases interleave and cover each other's stalls.
//
// LDS map (per work item):
//   sB[row][4][Q]   weighted operands of the item's local rows at the stage
//                   points: sqrt(w/2) d_x phi, sqrt(w/2) d_y phi,
//                   sqrt(w/2) d_z phi, sqrt(w) phi
//   sV[2][Q]        V at the stage points, two buffers for alternate stages
//   sPsi[f][FS]     (value, gradient) of the element's enrichment functions,
//                   component c of function f at f FS + c Q
//   sGeo[GEO][Q]    per-point geometry, one field after the other
//   sImg, sG, sEd   image centres, groups, enriched-function table
//   sLeaf, sPt, sGx leaf codes of the item, Gauss point digits, Gauss rule
//   sRow            local function of each item row (-1: padding)
template <int Q>
struct ContractLds {
    // row stride (doubles), odd: the MFMA operand reads (lane l at row l % 16,
    // point l / 16) then meet 16 distinct even bank pairs in each 16-lane
    // quarter of the wave; with an even stride (4 Q + 2) rows j and j + 8 met
    // on one bank pair and these reads carried every bank conflict of the
    // kernel (the row and enrichment phases, 16 consecutive points per unit,
    // have none)
    static constexpr int RS = 4 * Q + 1;
    static constexpr int FS = 4 * Q + 2;  // enrichment-function stride (doubles): offset banks
    static constexpr int GEO = 40;        // doubles of geometry per point
    static __host__ __device__ size_t bytes(int rows, int nfun, int nimg, int nleaf, int n3) {
        return sizeof(double) * ((size_t)rows * RS + 2 * (size_t)Q + (size_t)nfun * FS + (size_t)Q * GEO +
                                 (size_t)nimg * 3 + 2 * kMaxGauss) +
               sizeof(GroupDev) * kMaxGroups + sizeof(int32_t) * kMaxNloc +
               sizeof(uint32_t) * ((size_t)nleaf + n3 + rows + 16 + kMaxRowChunks + 4) + 64;
    }
};

constexpr int kContractThreads = 256;    // narrow work groups: 4 waves

// Enrichment slots of a wide work group (8 waves, 16-point stages): slot
// 4 p + s, s = lane / 16, of the p-th wave in the order of fewest tile pairs
// evaluates group slot[4 p + s] at the 16 stage points (-1: none).  Groups of
// one l fill waves of their own while the waves suffice, so each wave runs a
// single l branch of the evaluation, the heaviest (largest l) on the waves
// with the fewest MFMAs; otherwise the groups are packed by l.  One thread.
__device__ __forceinline__ void enrichment_slots(const PUFE_GLOBAL GroupDev *grp, int ngrp, int nw, int *slot) {
    int cnt[4] = {0, 0, 0, 0};
    for (int g = 0; g < ngrp; ++g) ++cnt[min(max(grp[g].l, 0), 3)];
    int need = 0;
    for (int l = 0; l < 4; ++l) need += (cnt[l] + 3) / 4;
    const bool own = need <= nw;
    for (int k = 0; k < 4 * nw; ++k) slot[k] = -1;
    int k = 0;
    for (int l = 3; l >= 0; --l) {
        if (own) k = (k + 3) & ~3;
        for (int g = 0; g < ngrp; ++g)
            if (min(max(grp[g].l, 0), 3) == l && k < 4 * nw) slot[k++] = g;
    }
}

constexpr int kWideWaves = 8;            // wide work groups (elements of more than 80 functions)
constexpr int kWideQ = 16;               // stage length of the wide work groups
static_assert(kMaxGroups <= 4 * kWideWaves, "every group has an enrichment slot in a wide work group");

// MFMAs of one stage for a wave owning NU tile pairs.  Every product sums
// k = 4 consecutive points of one operand component (lane l supplies row
// l % 16 at point 4 s4 + l / 16), five per pair and 4 points:
//   S   += u u^T,  H += u (V u)^T + g_x g_x^T + g_y g_y^T + g_z g_z^T,
// with u = sqrt(w) phi and g = sqrt(w/2) grad phi; V scales the B operand
// on load (one multiply per pair and step).
template <int Q, int NU>
__device__ __forceinline__ void mfma_stage(const double *__restrict__ sB, const double *__restrict__ sV,
                                           const int *pr_row, const int *pr_col, int r16, int k4, double4_t *accH,
                                           double4_t *accS) {
    constexpr int RS = ContractLds<Q>::RS;
#pragma unroll 1
    for (int s4 = 0; s4 < Q / 4; ++s4) {
        const int o = 4 * s4 + k4;
        const double vq = sV[o];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const double *ra = sB + (size_t)(pr_row[u] + r16) * RS + o;
            const double *rb = sB + (size_t)(pr_col[u] + r16) * RS + o;
            const double au = ra[3 * Q], bu = rb[3 * Q];
            const double ax = ra[0], bx = rb[0], ay = ra[Q], by = rb[Q], az = ra[2 * Q], bz = rb[2 * Q];
            accS[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bu, accS[u], 0, 0, 0);
            accH[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bu * vq, accH[u], 0, 0, 0);
            accH[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bx, accH[u], 0, 0, 0);
            accH[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, by, accH[u], 0, 0, 0);
            accH[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, bz, accH[u], 0, 0, 0);
        }
    }
}

// Tail pairs of a whole-element item: the last tile holds nt <= 8 real
// rows, so the pair (tile I, last tile) runs on v_mfma_f64_4x4x4f64, whose
// four blocks take the four 4-row groups of tile I against 4 tail columns
// (TG groups of 4 columns).  4x4x4 operand lane l = 16 k + 4 b + i holds
// A_b[i][k] (here row 4 b + i of tile I, i.e. row l % 16, at point k) and
// B_b[k][j] with j = l % 4 (the same tail column for every block); result
// lane l holds D_b[l / 16][l % 4], b = (l / 4) % 4.
template <int Q, int MT, int TG>
__device__ __forceinline__ void mfma_tail_stage(const double *__restrict__ sB, const double *__restrict__ sV,
                                                const int *tl_row, int tail_row0, int r16, int k4, int lane,
                                                double (*tH)[2], double (*tS)[2]) {
    constexpr int RS = ContractLds<Q>::RS;
#pragma unroll 1
    for (int s4 = 0; s4 < Q / 4; ++s4) {
        const int o = 4 * s4 + k4;
        const double vq = sV[o];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const double *ra = sB + (size_t)(tl_row[t] + r16) * RS + o;
            const double au = ra[3 * Q], ax = ra[0], ay = ra[Q], az = ra[2 * Q];
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const double *rb = sB + (size_t)(tail_row0 + 4 * g + (lane & 3)) * RS + o;
                const double bu = rb[3 * Q], bx = rb[0], by = rb[Q], bz = rb[2 * Q];
                tS[t][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(au, bu, tS[t][g], 0, 0, 0);
                tH[t][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(au, bu * vq, tH[t][g], 0, 0, 0);
                tH[t][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ax, bx, tH[t][g], 0, 0, 0);
                tH[t][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ay, by, tH[t][g], 0, 0, 0);
                tH[t][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(az, bz, tH[t][g], 0, 0, 0);
            }
        }
    }
}

template <int Q, int TG>
__device__ __forceinline__ void mfma_tail_dispatch(int mt, const double *sB, const double *sV, const int *tl_row,
                                                   int tail_row0, int r16, int k4, int lane, double (*tH)[2],
                                                   double (*tS)[2]) {
    switch (mt) {
        case 3: mfma_tail_stage<Q, 3, TG>(sB, sV, tl_row, tail_row0, r16, k4, lane, tH, tS); break;
        case 2: mfma_tail_stage<Q, 2, TG>(sB, sV, tl_row, tail_row0, r16, k4, lane, tH, tS); break;
        case 1: mfma_tail_stage<Q, 1, TG>(sB, sV, tl_row, tail_row0, r16, k4, lane, tH, tS); break;
        default: break;
    }
}

// NW waves per work group: 4 (narrow: up to 4 tile pairs per wave, two
// work groups per CU where LDS allows) or 8 (wide: up to 5 pairs per wave,
// one work group of 2 waves per SIMD, for the large row and column blocks of
// elements of many functions, which then evaluate their enrichment functions
// and rows for fewer items).
template <int Q, int LMAX, int NW = 4, bool GEN = false>
__device__ __forceinline__ void contract_f64_item(
    const KParams &kpg, const ItemDev &it, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial, double *smem,
    int rot) {
    constexpr int RS = ContractLds<Q>::RS;
    constexpr int FS = ContractLds<Q>::FS;
    constexpr int GEO = ContractLds<Q>::GEO;
    constexpr int NT = 64 * NW;
    constexpr int NUMAX = NW == 4 ? 4 : 5;   // tile pairs per wave
    const KLocal kp = load_klocal(kpg);
    // The table pointers of a batched launch are read from memory, so the
    // compiler cannot tell that they address global memory; typed as such,
    // their loads are global rather than flat instructions (a flat load in
    // flight would also hold up every wait on LDS traffic).
    const PUFE_GLOBAL ElemDev *gElems = (const PUFE_GLOBAL ElemDev *)elems;
    const PUFE_GLOBAL GroupDev *gGroups = (const PUFE_GLOBAL GroupDev *)groups;
    const PUFE_GLOBAL double *gImg = (const PUFE_GLOBAL double *)img;
    const PUFE_GLOBAL int32_t *gEdof = (const PUFE_GLOBAL int32_t *)edof;
    const PUFE_GLOBAL uint32_t *gLeaves = (const PUFE_GLOBAL uint32_t *)leaves;
    const PUFE_GLOBAL double *gV = (const PUFE_GLOBAL double *)V;
    PUFE_GLOBAL double *gPartial = (PUFE_GLOBAL double *)partial;
    const PUFE_GLOBAL ElemDev &el = gElems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun;
    const bool diag = it.I0 == it.J0;
    const int nrow = 16 * (diag ? it.nI : it.nI + it.nJ);
    const int img0 = ngrp > 0 ? gGroups[el.grp_off].img_off : 0;
    const int nimg = ngrp > 0 ? gGroups[el.grp_off + ngrp - 1].img_off + gGroups[el.grp_off + ngrp - 1].nimg - img0 : 0;
    // image weights of a Bloch-periodic enrichment, indexed like sImg
    const double *wimg = (GEN && kp.wimg) ? kp.wimg + img0 : nullptr;
    const uint32_t n3 = (uint32_t)kp.n3, n = (uint32_t)kp.n;
    double *sB = smem;                                        // [nrow][RS]
    double *sV = sB + (size_t)nrow * RS;                      // [2][Q], alternate stages
    double *sPsi = sV + 2 * Q;                                // [nfun][FS]
    double *sGeo = sPsi + (size_t)nfun * FS;                  // [GEO][Q]
    double *sImg = sGeo + (size_t)Q * GEO;
    double *sGx = sImg + 3 * (size_t)nimg, *sGs = sGx + kMaxGauss;   // square roots of the 1D Gauss weights
    GroupDev *sG = (GroupDev *)(sGs + kMaxGauss);
    int32_t *sEd = (int32_t *)(sG + kMaxGroups);
    uint32_t *sLeaf = (uint32_t *)(sEd + kMaxNloc);
    uint32_t *sPt = sLeaf + (it.leaf_e - it.leaf_b);
    int *sRow = (int *)(sPt + n3);
    int *sCS = sRow + nrow;   // [9] PU corner starts in sEd
    int *sChunk = sCS + 16;   // [kMaxRowChunks] enriched-row chunks of a partial item, and their count
    int *sNChunk = sChunk + kMaxRowChunks;
    int *sSlot = sNChunk + 4;   // [4 NW] enrichment slots of a wide work group (beyond ContractLds::bytes)
    constexpr bool kSlots = NW == 8 && Q == 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q_begin = it.leaf_b * (int64_t)n3, q_end = it.leaf_e * (int64_t)n3;
    const uint32_t nli = (uint32_t)(q_end - q_begin);
    const int ti0 = it.I0, tj0 = it.J0;
    for (int k = tid; k < nloc - nfe; k += NT) sEd[k] = gEdof[el.edof_off + k];
    // an item holding every row of its element evaluates them in groups that
    // share a point's geometry (FE functions by (a2, a3), enriched ones by
    // PU corner); other items take one row at a time
    const bool whole = diag && ti0 == 0 && 16 * it.nI >= nloc;
    corner_starts(gEdof + el.edof_off, nloc - nfe, sCS, tid, NT);
    // local functions of a partial item: rows [lo0, hi0) then, off the
    // diagonal, [lo1, hi1), at LDS rows 0 and 16 nI
    const int lo0 = 16 * ti0, hi0 = min(16 * (ti0 + it.nI), nloc);
    const int lo1 = diag ? 0 : 16 * tj0, hi1 = diag ? 0 : min(16 * (tj0 + it.nJ), nloc);
    for (int g = tid; g < ngrp; g += NT) {
        const PUFE_GLOBAL GroupDev &Gg = gGroups[el.grp_off + g];
        GroupDev G;
        G.atom = Gg.atom;
        G.desc = Gg.desc;
        G.l = Gg.l;
        G.fbase = Gg.fbase;
        G.img_off = Gg.img_off - img0;   // rebased onto sImg
        G.nimg = Gg.nimg;
        G.nspl = Gg.nspl;
        G.spl_off = Gg.spl_off;
        G.a = Gg.a;
        G.rc = Gg.rc;
        sG[g] = G;
    }
    if (kSlots && tid == 0) enrichment_slots(gGroups + el.grp_off, ngrp, NW, sSlot);
    for (int k = tid; k < 3 * nimg; k += NT) sImg[k] = gImg[3 * (size_t)img0 + k];
    for (int64_t k = tid; k < it.leaf_e - it.leaf_b; k += NT) sLeaf[k] = gLeaves[it.leaf_b + k];
    for (uint32_t j = tid; j < n3; j += NT) sPt[j] = (j % n) | (((j / n) % n) << 8) | ((j / (n * n)) << 16);
    for (int r = tid; r < nrow; r += NT) {
        const int a = (diag || r < 16 * it.nI) ? 16 * ti0 + r : 16 * tj0 + (r - 16 * it.nI);
        sRow[r] = a < nloc ? a : -1;
    }
    // rows past the element's functions are the tail of the last tile
    const int nreal = diag ? min(nrow, nloc - 16 * ti0) : 16 * it.nI + min(16 * it.nJ, nloc - 16 * tj0);
    for (int k = tid; k < (nrow - nreal) * RS; k += NT) sB[(size_t)nreal * RS + k] = 0.0;
    if (tid < kp.n) {
        sGx[tid] = kpg.gx[tid];
        sGs[tid] = sqrt(kpg.gw[tid]);
    }
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};

    // tile pairs of this item, round-robin over the four waves starting at
    // wave rot: when the pairs do not divide by four, work groups sharing a
    // CU then load its four SIMDs' MFMA units unevenly in different ways
    // rather than all on the same SIMDs
    //
    // Whole-element items whose last tile holds at most 8 real rows take the
    // pairs (I, last tile) as tail pairs on the 4x4x4 MFMA (a quarter or half
    // the cost of a full pair), handed one by one to the least loaded wave;
    // the remaining pairs are the full pairs of the other tiles.
    const int T = (nloc + 15) / 16;
    const int ntail = nloc - 16 * (T - 1);
    // (compiled for enrichments up to l = 1 only: with l up to 3 the extra
    // accumulators would push the kernel into register spills)
    constexpr bool kTail = LMAX <= 1 && NW == 4;
    const int tg = (kTail && whole && T >= 2) ? (ntail <= 4 ? 1 : (ntail <= 8 ? 2 : 0)) : 0;
    const int npairs = tg ? (T - 1) * T / 2 : (diag ? it.nI * (it.nI + 1) / 2 : it.nI * it.nJ);
    const int vw = (wave - rot + NW) % NW;
    const int nu = npairs > vw ? (npairs - vw + NW - 1) / NW : 0;   // pairs of this wave (uniform)
    constexpr int MAXT = 3;   // tail pairs per wave (at most 5 tail pairs per item)
    int mt = 0, tl_row[MAXT] = {0, 0, 0}, tl_I[MAXT] = {0, 0, 0};
    if (tg) {
        // loads in quarter pairs; ties go to the higher virtual wave, which
        // holds fewer full pairs
        int l0 = 4 * (npairs > 0 ? (npairs + 3) / 4 : 0), l1 = 4 * (npairs > 1 ? (npairs + 2) / 4 : 0);
        int l2 = 4 * (npairs > 2 ? (npairs + 1) / 4 : 0), l3 = 4 * (npairs > 3 ? npairs / 4 : 0);
        for (int I = 0; I < T; ++I) {
            int best = 3, lb = l3;
            if (l2 < lb) { best = 2; lb = l2; }
            if (l1 < lb) { best = 1; lb = l1; }
            if (l0 < lb) { best = 0; lb = l0; }
            l0 += best == 0 ? tg : 0;
            l1 += best == 1 ? tg : 0;
            l2 += best == 2 ? tg : 0;
            l3 += best == 3 ? tg : 0;
            if (best == vw && mt < MAXT) {
#pragma unroll
                for (int t = 0; t < MAXT; ++t)
                    if (t == mt) {
                        tl_row[t] = 16 * I;
                        tl_I[t] = I;
                    }
                ++mt;
            }
        }
    }
    double tH[MAXT][2], tS[MAXT][2];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) tH[t][0] = tH[t][1] = tS[t][0] = tS[t][1] = 0.0;
    int pr_row[NUMAX], pr_col[NUMAX], pr_I[NUMAX], pr_J[NUMAX];
#pragma unroll
    for (int u = 0; u < NUMAX; ++u) {
        const int pidx = vw + NW * u;
        pr_row[u] = pr_col[u] = pr_I[u] = pr_J[u] = 0;
        if (u < nu) {
            int a, b;
            if (diag) {  // enumerate (a <= b) column by column
                b = 0;
                while ((b + 1) * (b + 2) / 2 <= pidx) ++b;
                a = pidx - b * (b + 1) / 2;
                pr_row[u] = 16 * a;
                pr_col[u] = 16 * b;
                pr_I[u] = ti0 + a;
                pr_J[u] = ti0 + b;
            } else {
                a = pidx % it.nI;
                b = pidx / it.nI;
                pr_row[u] = 16 * a;
                pr_col[u] = 16 * (it.nI + b);
                pr_I[u] = ti0 + a;
                pr_J[u] = tj0 + b;
            }
        }
    }
    double4_t accH[NUMAX], accS[NUMAX];
#pragma unroll
    for (int u = 0; u < NUMAX; ++u) {
        accH[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
        accS[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
    }
    const int r16 = lane & 15, k4 = lane >> 4;
    // the last Q threads build the geometry (a wide work group: the last 16
    // lanes of its wave of the fewest-MFMA order's fourth place, whose slots
    // hold the lightest groups, l = 0 where the element has four l); V is read
    // one stage ahead
    const int gq = kSlots ? (vw == NW - 4 ? lane - (64 - Q) : -1) : tid - (NT - Q);
    double v = (gq >= 0 && (uint32_t)gq < nli) ? gV[q_begin + gq] : 0.0;
    // phase 1 of the stage starting at lbx: enrichment functions (eq. Psi,
    // f(R) = 1) and geometry, and V of that stage into the buffer vb
    auto phase1 = [&](uint32_t lbx, double *vb) {
        if (gq >= 0) {
            const double vn = (lbx + Q + gq < nli) ? gV[q_begin + lbx + Q + gq] : 0.0;
            double xi[3], sw;
            item_point(kp, sLeaf, sPt, sGx, sGs, lbx + gq, nli, n3, xi, &sw);
            point_geometry<Q>(kp, org, xi, sw, sGeo + gq);
            vb[gq] = v;
            v = vn;
        }
        auto eval = [&](int g, int q) {
            const GroupDev &G = sG[g];
            double xi[3], sw, x[3];
            item_point(kp, sLeaf, sPt, sGx, sGs, lbx + q, nli, n3, xi, &sw);
            point_position(kp, org, xi, x);
            group_eval_upto<LMAX, Q, FS, GEN>(G, sImg, kp.spl, wimg, x, sPsi + (size_t)G.fbase * FS + q);
        };
        if constexpr (kSlots) {
            // one pass: the wave's slot of 16 lanes, waves taken by fewest tile pairs
            const int g = sSlot[4 * (NW - 1 - vw) + (lane >> 4)];
            if (g >= 0) eval(g, lane & 15);
        } else {
            for (int idx = tid; idx < ngrp * Q; idx += NT) {
                const int g = idx / Q;
                eval(g, idx - g * Q);
            }
        }
    };
    __syncthreads();
    // FE functions in the item's rows (grouped by (a2, a3), filtered on store)
    const int nfu = (whole || lo0 < nfe || (!diag && lo1 < nfe)) ? fe_units(kp.p) : 0;
    // (the one-pass widening pays on the wide work groups only: 0.8 % slower
    // on the narrow ones of the LiH-like cell)
    if (!whole && tid == 0) row_chunks(sCS, nfe, lo0, hi0, lo1, hi1, Q, NT, NW == 8 ? nfu : -1, sChunk, sNChunk);
    if (nli > 0) phase1(0, sV);
    __syncthreads();

    for (uint32_t lb = 0, st = 0; lb < nli; lb += Q, st ^= 1) {
        double *sVc = sV + st * Q;
        // ---- phase 2: weighted local basis rows (eq. pufebasis) of the
        // item's functions (the padding rows past them stay zero)
        if (whole) {
            for (int idx = tid; idx < nfu * Q; idx += NT) {
                const int u = idx / Q, q = idx - u * Q;
                double *o = sB + q;
                auto put = [&](int a, double x, double y, double z, double w) {
                    double *r = o + (size_t)a * RS;
                    r[0] = x;
                    r[Q] = y;
                    r[2 * Q] = z;
                    r[3 * Q] = w;
                };
                fe_unit_any<Q, false, GEN>(kp, sGeo + q, u, put);
            }
            for (int idx = tid; idx < 8 * Q; idx += NT) {
                const int c = idx / Q, q = idx - c * Q;
                double *o = sB + q;
                auto put = [&](int a, double x, double y, double z, double w) {
                    double *r = o + (size_t)a * RS;
                    r[0] = x;
                    r[Q] = y;
                    r[2 * Q] = z;
                    r[3 * Q] = w;
                };
                pu_unit<Q, FS>(kp, sGeo + q, sPsi + q, sEd, c, sCS[c], sCS[c + 1], nfe, put);
            }
        } else {
            // partial items: the same geometry-sharing groups, the enriched
            // ones cut into the chunks of the item's rows (row_chunks)
            const int nch = *sNChunk;
            for (int idx = tid; idx < (nfu + nch) * Q; idx += NT) {
                const int u = idx / Q, q = idx - u * Q;
                double *o = sB + q;
                auto put = [&](int a, double x, double y, double z, double w) {
                    int r;
                    if (a >= lo0 && a < hi0) r = a - lo0;
                    else if (a >= lo1 && a < hi1) r = 16 * it.nI + (a - lo1);
                    else return;
                    double *rr = o + (size_t)r * RS;
                    rr[0] = x;
                    rr[Q] = y;
                    rr[2 * Q] = z;
                    rr[3 * Q] = w;
                };
                if (u < nfu) {
                    fe_unit_any<Q, false, GEN>(kp, sGeo + q, u, put);
                } else {
                    const int ch = sChunk[u - nfu];
                    pu_unit<Q, FS>(kp, sGeo + q, sPsi + q, sEd, ch & 7, (ch >> 3) & 1023, ch >> 13, nfe, put);
                }
            }
        }
        __syncthreads();
        // ---- phase 3: the MFMAs of this stage (V from its buffer), then
        // phase 1 of the next stage, in one barrier interval: phase 3 reads
        // only the rows and V, phase 1 writes the enrichment table, the
        // geometry and the other V buffer
        switch (nu) {
            case 5: if (NUMAX >= 5) mfma_stage<Q, 5>(sB, sVc, pr_row, pr_col, r16, k4, accH, accS); break;
            case 4: mfma_stage<Q, 4>(sB, sVc, pr_row, pr_col, r16, k4, accH, accS); break;
            case 3: mfma_stage<Q, 3>(sB, sVc, pr_row, pr_col, r16, k4, accH, accS); break;
            case 2: mfma_stage<Q, 2>(sB, sVc, pr_row, pr_col, r16, k4, accH, accS); break;
            case 1: mfma_stage<Q, 1>(sB, sVc, pr_row, pr_col, r16, k4, accH, accS); break;
            default: break;
        }
        if (tg == 1)
            mfma_tail_dispatch<Q, 1>(mt, sB, sVc, tl_row, 16 * (T - 1), r16, k4, lane, tH, tS);
        else if (tg == 2)
            mfma_tail_dispatch<Q, 2>(mt, sB, sVc, tl_row, 16 * (T - 1), r16, k4, lane, tH, tS);
        if (lb + Q < nli) phase1(lb + Q, sV + (st ^ 1) * Q);
        __syncthreads();
    }
    // ---- partial tiles, row-major 16x16.  FP64 16x16x4 accumulator layout:
    // register r of lane l holds D[(l / 16) + 4 r][l % 16].
    const int64_t P = (int64_t)T * (T + 1) / 2;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        if (t >= mt) continue;
        const int64_t pidx = (int64_t)(T - 1) * T / 2 + tl_I[t];
        PUFE_GLOBAL double *dst = gPartial + (el.part_base + (int64_t)it.chunk * P + pidx) * 512;
        const int row = 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
        for (int g = 0; g < 2; ++g)
            if (g < tg) {
                dst[row * 16 + 4 * g + (lane & 3)] = tH[t][g];
                dst[256 + row * 16 + 4 * g + (lane & 3)] = tS[t][g];
            }
        // columns past the tail groups hold no function: zeros
        const int w = 16 - 4 * tg;
        for (int e = lane; e < 16 * w; e += 64) {
            const int zr = e / w, zc = 4 * tg + e % w;
            dst[zr * 16 + zc] = 0.0;
            dst[256 + zr * 16 + zc] = 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < NUMAX; ++u) {
        if (u >= nu) continue;
        const int64_t pidx = (int64_t)pr_J[u] * (pr_J[u] + 1) / 2 + pr_I[u];
        PUFE_GLOBAL double *dst = gPartial + (el.part_base + (int64_t)it.chunk * P + pidx) * 512;
        const int j = lane & 15, i0 = lane >> 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dst[(i0 + 4 * r) * 16 + j] = accH[u][r];
            dst[256 + (i0 + 4 * r) * 16 + j] = accS[u][r];
        }
    }
}

// One work group per work item.
template <int Q, int LMAX, bool GEN>
__global__ __launch_bounds__(kContractThreads) __attribute__((amdgpu_waves_per_eu(2))) void contract_f64_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const ItemDev it = items[blockIdx.x];
    contract_f64_item<Q, LMAX, 4, GEN>(kp, it, elems, groups, img, edof, leaves, V, partial, smem,
                               (blockIdx.x ^ (blockIdx.x >> 3) ^ (blockIdx.x >> 5) ^ (blockIdx.x >> 8)) & 3);
}

// Persistent form: a fixed grid of work groups pulls items (of several
// problems) from one queue, largest first; every item writes its own partial
// slots, so the result does not depend on which group ran it.
template <int Q, int LMAX, bool GEN>
__global__ __launch_bounds__(kContractThreads) __attribute__((amdgpu_waves_per_eu(2))) void contract_f64_persistent(const CtxDev *__restrict__ ctxs,
                                                                            const ItemDev *__restrict__ items,
                                                                            int n_items, int *__restrict__ counter) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= n_items) break;
        const ItemDev it = items[idx];
        const CtxDev &c = ctxs[it.ctx];
        contract_f64_item<Q, LMAX, 4, GEN>(c.kp, it, c.elems, c.groups, c.img, c.edof, c.leaves, c.V, c.partial, smem,
                                           idx & 3);
    }
}

// Wide work groups (8 waves, one per CU) for the items of elements of more
// than 80 functions.
template <int LMAX, bool GEN>
__global__ __launch_bounds__(64 * kWideWaves) __attribute__((amdgpu_waves_per_eu(2))) void contract_f64_wide_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const ItemDev it = items[blockIdx.x];
    contract_f64_item<kWideQ, LMAX, kWideWaves, GEN>(kp, it, elems, groups, img, edof, leaves, V, partial, smem,
                                                     blockIdx.x & 7);
}

template <int LMAX, bool GEN>
__global__ __launch_bounds__(64 * kWideWaves) __attribute__((amdgpu_waves_per_eu(2))) void contract_f64_wide_persistent(
    const CtxDev *__restrict__ ctxs, const ItemDev *__restrict__ items, int n_items, int *__restrict__ counter) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= n_items) break;
        const ItemDev it = items[idx];
        const CtxDev &c = ctxs[it.ctx];
        contract_f64_item<kWideQ, LMAX, kWideWaves, GEN>(c.kp, it, c.elems, c.groups, c.img, c.edof, c.leaves, c.V,
                                                         c.partial, smem, idx & 7);
    }
}

__global__ void reset_counter_kernel(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// ------------------------------------------------------ K-chunk reduction

// Sum of the K-chunk partial tiles of one (element, tile pair), in chunk
// order, into the chunk-0 slot; elements of one chunk are not listed.
__device__ __forceinline__ void chunk_reduce_tile(const ElemDev &el, int pidx, double *__restrict__ partial) {
    const int T = (el.nloc + 15) / 16;
    const int64_t P = (int64_t)T * (T + 1) / 2;
    double *dst = partial + (el.part_base + pidx) * 512;
    for (int k = threadIdx.x; k < 512; k += blockDim.x) {
        double acc = 0.0;
        int c = 0;
        // four chunks in flight, added in chunk order
        for (; c + 4 <= el.nchunk; c += 4) {
            const double v0 = dst[(int64_t)c * P * 512 + k], v1 = dst[(int64_t)(c + 1) * P * 512 + k];
            const double v2 = dst[(int64_t)(c + 2) * P * 512 + k], v3 = dst[(int64_t)(c + 3) * P * 512 + k];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; c < el.nchunk; ++c) acc += dst[(int64_t)c * P * 512 + k];
        dst[k] = acc;
    }
}

__global__ __launch_bounds__(256) void chunk_reduce_kernel(const ElemDev *__restrict__ elems,
                                                           const int2 *__restrict__ list,
                                                           double *__restrict__ partial) {
    const int2 ep = list[blockIdx.x];
    chunk_reduce_tile(elems[ep.x], ep.y, partial);
}

__global__ __launch_bounds__(256) void chunk_reduce_batch_kernel(const CtxDev *__restrict__ ctxs,
                                                                 const int4 *__restrict__ list) {
    const int4 ce = list[blockIdx.x];
    const CtxDev &c = ctxs[ce.x];
    chunk_reduce_tile(c.elems[ce.y], ce.z, c.partial);
}

// -------------------------------------------------------------- scatter

__global__ void fill_zero_kernel(double *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

__global__ void fill_zero_f32_kernel(float *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0f;
}

// Phase table z[k][t] = exp(2 pi i kappa_k . dn), dn = (t % 3, t / 3 % 3, t / 9) - 1:
// the factor conj(p_a) p_b of a local pair whose corners differ by the
// lattice shift dn (the Bloch phase factors at the cell boundary).
__device__ __forceinline__ void phase_entry(const KPoints &kps, int idx, double2 *__restrict__ z) {
    const int k = idx / 27, t = idx % 27;
    const int dn[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
    double sn, cs;
    sincos(2.0 * M_PI * (kps.kap[k][0] * dn[0] + kps.kap[k][1] * dn[1] + kps.kap[k][2] * dn[2]), &sn, &cs);
    z[idx] = make_double2(cs, sn);
}

__global__ void phase_table_kernel(const KPoints kps, double2 *__restrict__ z) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kps.nk * 27) return;
    phase_entry(kps, idx, z);
}

// Zero fill of the H and S outputs of an assembly (nw 8-byte words each; S
// may be null; zero bits serve every output type) and, in the first work
// group, the phase table of its k-points: one launch ahead of the scatter.
__global__ void prepare_outputs_kernel(double *__restrict__ H, double *__restrict__ S, int64_t nw, const KPoints kps,
                                       double2 *__restrict__ z) {
    if (blockIdx.x == 0)
        for (int idx = threadIdx.x; idx < kps.nk * 27; idx += blockDim.x) phase_entry(kps, idx, z);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride) {
        H[i] = 0.0;
        if (S) S[i] = 0.0;
    }
}

// One upper tile pair (I, J) of one element: each thread owns one entry
// (a, b), a <= b, sums its K-chunk partials in chunk order, and for every
// k-point adds conj(p_a) p_b H_e[a][b] at (g_a, g_b) and the conjugate at
// (g_b, g_a).  The elements of one launch share no vertex (one colour), so
// no two threads of a launch touch the same entry.
__device__ __forceinline__ void scatter_tile(const KParams &kp, const ElemDev &el, int pidx,
                                             const int32_t *__restrict__ edof, const double *__restrict__ partial,
                                             const double2 *__restrict__ z, int nk, int out_dtype,
                                             void *__restrict__ Hout, void *__restrict__ Sout, int64_t nnz) {
    const int nloc = el.nloc;
    int J = 0;
    while ((J + 1) * (J + 2) / 2 <= pidx) ++J;
    const int I = pidx - J * (J + 1) / 2;
    const int i = (int)(threadIdx.x >> 4), j = (int)(threadIdx.x & 15);
    const int a = 16 * I + i, b = 16 * J + j;
    if (a >= nloc || b >= nloc || a > b) return;
    const int T = (nloc + 15) / 16;
    const int64_t P = (int64_t)T * (T + 1) / 2;
    // the K-chunk partials were summed into the chunk-0 slot
    const double *src = partial + (el.part_base + pidx) * 512;
    const double h = src[i * 16 + j], s = src[256 + i * 16 + j];
    int ca, sa, cb, sb;
    local_slot(el, edof, kp.p, a, &ca, &sa);
    local_slot(el, edof, kp.p, b, &cb, &sb);
    const int64_t oab = el.blk[ca * 8 + cb] + (int64_t)sa * el.bw[cb] + sb;
    const int64_t oba = el.blk[cb * 8 + ca] + (int64_t)sb * el.bw[ca] + sa;
    int t = 0;
    for (int d = 2; d >= 0; --d) {
        const int dn = ((el.shifts >> (3 * cb + d)) & 1) - ((el.shifts >> (3 * ca + d)) & 1);
        t = 3 * t + (dn + 1);
    }
    if (out_dtype == 0) {
        // complex128: four k-points at a time, all loads before the stores
        // (the k-point arrays are disjoint), so their latencies overlap
        double2 *H2 = (double2 *)Hout, *S2 = (double2 *)Sout;
        for (int k0 = 0; k0 < nk; k0 += 4) {
            double2 zk[4], hab[4], hba[4], sab[4], sba[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k0 + u >= nk) break;
                const int64_t base = (int64_t)(k0 + u) * nnz;
                zk[u] = z[(k0 + u) * 27 + t];
                hab[u] = H2[base + oab];
                if (a != b) hba[u] = H2[base + oba];
                if (Sout) {
                    sab[u] = S2[base + oab];
                    if (a != b) sba[u] = S2[base + oba];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k0 + u >= nk) break;
                const int64_t base = (int64_t)(k0 + u) * nnz;
                const double cr = zk[u].x, ci = zk[u].y;
                H2[base + oab] = make_double2(hab[u].x + cr * h, hab[u].y + ci * h);
                if (a != b) H2[base + oba] = make_double2(hba[u].x + cr * h, hba[u].y - ci * h);
                if (Sout) {
                    S2[base + oab] = make_double2(sab[u].x + cr * s, sab[u].y + ci * s);
                    if (a != b) S2[base + oba] = make_double2(sba[u].x + cr * s, sba[u].y - ci * s);
                }
            }
        }
        return;
    }
    for (int k = 0; k < nk; ++k) {
        const double2 zz = z[k * 27 + t];
        const double cr = zz.x, ci = zz.y;
        if (out_dtype == 1) {
            float *H = (float *)Hout + 2 * (int64_t)k * nnz;
            H[2 * oab] += (float)(cr * h);
            H[2 * oab + 1] += (float)(ci * h);
            if (a != b) {
                H[2 * oba] += (float)(cr * h);
                H[2 * oba + 1] -= (float)(ci * h);
            }
            if (Sout) {
                float *S = (float *)Sout + 2 * (int64_t)k * nnz;
                S[2 * oab] += (float)(cr * s);
                S[2 * oab + 1] += (float)(ci * s);
                if (a != b) {
                    S[2 * oba] += (float)(cr * s);
                    S[2 * oba + 1] -= (float)(ci * s);
                }
            }
        } else {
            double *H = (double *)Hout + (int64_t)k * nnz;
            H[oab] += h;
            if (a != b) H[oba] += h;
            if (Sout) {
                double *S = (double *)Sout + (int64_t)k * nnz;
                S[oab] += s;
                if (a != b) S[oba] += s;
            }
        }
    }
}

__global__ __launch_bounds__(256) void scatter_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                      const int2 *__restrict__ list,
                                                      const int32_t *__restrict__ edof,
                                                      const double *__restrict__ partial,
                                                      const double2 *__restrict__ z, int nk, int out_dtype,
                                                      void *__restrict__ Hout, void *__restrict__ Sout, int64_t nnz) {
    const int2 ep = list[blockIdx.x];
    scatter_tile(kp, elems[ep.x], ep.y, edof, partial, z, nk, out_dtype, Hout, Sout, nnz);
}

// Batched scatter of one colour: (problem, element, tile pair) of several
// problems, each into its own output.
__global__ __launch_bounds__(256) void scatter_batch_kernel(const CtxDev *__restrict__ ctxs,
                                                            const int4 *__restrict__ list,
                                                            const double2 *__restrict__ z, int nk,
                                                            int out_dtype) {
    const int4 ce = list[blockIdx.x];
    const CtxDev &c = ctxs[ce.x];
    scatter_tile(c.kp, c.elems[ce.y], ce.z, c.edof, c.partial, z, nk, out_dtype, c.H, c.S, c.nnz);
}

// Element matrices of one element (full, mirrored), from its partials.
__global__ void elem_matrices_kernel(const ElemDev *__restrict__ elems, int64_t e,
                                     const double *__restrict__ partial, double *__restrict__ He,
                                     double *__restrict__ Se, int ld) {
    const ElemDev &el = elems[e];
    const int nloc = el.nloc, T = (nloc + 15) / 16;
    const int64_t P = (int64_t)T * (T + 1) / 2;
    for (int64_t idx = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; idx < (int64_t)nloc * nloc;
         idx += (int64_t)blockDim.x * gridDim.x) {
        int a = (int)(idx / nloc), b = (int)(idx % nloc);
        int lo = a < b ? a : b, hi = a < b ? b : a;
        int I = lo / 16, J = hi / 16, i = lo % 16, j = hi % 16;
        int64_t pidx = (int64_t)J * (J + 1) / 2 + I;
        const double *src = partial + (el.part_base + pidx) * 512;   // chunk sums (reduced)
        He[(int64_t)a * ld + b] = src[i * 16 + j];
        Se[(int64_t)a * ld + b] = src[256 + i * 16 + j];
    }
}

// BSR values (C128 or real) -> dense complex n x n, row-major.
__global__ void bsr_to_dense_kernel(int64_t nnzb, const int32_t *__restrict__ brow,
                                    const int32_t *__restrict__ bcol, const int64_t *__restrict__ bval_off,
                                    const int64_t *__restrict__ dof_off, const void *__restrict__ src, int dtype,
                                    int64_t n, double *__restrict__ dense) {
    for (int64_t blk = blockIdx.x; blk < nnzb; blk += gridDim.x) {
        const int64_t v = brow[blk], w = bcol[blk];
        const int64_t r0 = dof_off[v], c0 = dof_off[w];
        const int bc = (int)(dof_off[w + 1] - c0);
        const int64_t cnt = bval_off[blk + 1] - bval_off[blk];
        for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
            const int64_t r = t / bc, c = t % bc;
            const int64_t src_i = bval_off[blk] + t;
            const int64_t dst = ((r0 + r) * n + (c0 + c)) * 2;
            if (dtype == 0) {
                dense[dst] = ((const double *)src)[2 * src_i];
                dense[dst + 1] = ((const double *)src)[2 * src_i + 1];
            } else {
                dense[dst] = ((const double *)src)[src_i];
                dense[dst + 1] = 0.0;
            }
        }
    }
}

// ------------------------------------------- allocation-free workspace
//
// The workspace of pufe_assemble_noalloc: the phase table and the K-chunk
// partial tiles of one assembly, in a fixed array that the code object
// brings with it (each GPU holds its own copy for the life of the process).
// In host code `scratch` is only a host-side stand-in for the symbol: kernels
// get the device address that hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

hipError_t scratch_address(int device, double **ptr) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// ------------------------------------------------------------- launchers

#define PUFE_HIP(x)                              \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return e_;         \
    } while (0)

hipError_t launch_aq_geom(const KParams &kp, int64_t nel, const double *pos, int n_atoms, const double *L,
                          int max_level, double dist, int64_t *count, const int64_t *off, uint32_t *out,
                          int32_t *leaf_elem, hipStream_t st) {
    int blocks = (int)((nel + 127) / 128);
    hipLaunchKernelGGL(aq_geom_kernel, dim3(blocks), dim3(128), 0, st, kp, nel, pos, n_atoms, L[0], L[1], L[2],
                       max_level, dist * dist, count, off, out, leaf_elem);
    return hipGetLastError();
}

hipError_t launch_scan(const int64_t *in, int64_t n, int64_t *off, hipStream_t st) {
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, in, n, off);
    return hipGetLastError();
}

hipError_t launch_qp_export(const KParams &kp, int64_t n_leaves, const uint32_t *leaves, const int32_t *leaf_elem,
                            double *xyz, double *w, hipStream_t st) {
    int64_t nq = n_leaves * kp.n3;
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(qp_export_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, kp, n_leaves,
                       leaves, leaf_elem, xyz, w);
    return hipGetLastError();
}

hipError_t launch_elem_qp_offset(const KParams &kp, int64_t nel, const int64_t *leaf_off, int64_t *qp_off,
                                 hipStream_t st) {
    hipLaunchKernelGGL(elem_qp_offset_kernel, dim3((unsigned)((nel + 256) / 256)), dim3(256), 0, st, kp, nel,
                       leaf_off, qp_off);
    return hipGetLastError();
}

size_t contract_lds_bytes(int q, int rows, int nfun, int nimg, int nleaf, int n3) {
    switch (q) {
        case 32: return ContractLds<32>::bytes(rows, nfun, nimg, nleaf, n3);
        case 24: return ContractLds<24>::bytes(rows, nfun, nimg, nleaf, n3);
        default: return ContractLds<16>::bytes(rows, nfun, nimg, nleaf, n3);
    }
}

bool contract_q_supported(int q) { return q == 16 || q == 24 || q == 32; }

hipError_t launch_contract_f64(int q, int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items,
                               const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                               const uint32_t *leaves, const double *V, double *partial, size_t lds,
                               hipStream_t st) {
    if (n_items == 0) return hipSuccess;
#define PUFE_PLAIN(QQ, LL, TT)                                                                                   \
    hipLaunchKernelGGL((contract_f64_kernel<QQ, LL, TT>), dim3(n_items), dim3(kContractThreads), lds, st, kp, items, \
                       elems, groups, img, edof, leaves, V, partial)
#define PUFE_PLAIN_Q(QQ)                       \
    do {                                       \
        if (gen) PUFE_PLAIN(QQ, 3, true);      \
        else if (lmax <= 1) PUFE_PLAIN(QQ, 1, false); \
        else PUFE_PLAIN(QQ, 3, false);         \
    } while (0)
    if (q == 32) PUFE_PLAIN_Q(32);
    else if (q == 24) PUFE_PLAIN_Q(24);
    else PUFE_PLAIN_Q(16);
#undef PUFE_PLAIN_Q
#undef PUFE_PLAIN
    return hipGetLastError();
}

// Dynamic LDS above the default limit must be enabled per kernel before any
// launch (and before any graph capture).
hipError_t init_contract_attributes() {
    // analytic radials and Lagrange elements (l <= 1, l <= 3), and the general
    // variant (tabulated radials, serendipity elements; l <= 3)
    const void *ks[] = {(const void *)contract_f64_kernel<16, 1, false>, (const void *)contract_f64_kernel<16, 3, false>,
                        (const void *)contract_f64_kernel<16, 3, true>, (const void *)contract_f64_kernel<24, 1, false>,
                        (const void *)contract_f64_kernel<24, 3, false>, (const void *)contract_f64_kernel<24, 3, true>,
                        (const void *)contract_f64_kernel<32, 1, false>, (const void *)contract_f64_kernel<32, 3, false>,
                        (const void *)contract_f64_kernel<32, 3, true>,
                        (const void *)contract_f64_persistent<16, 1, false>, (const void *)contract_f64_persistent<16, 3, false>,
                        (const void *)contract_f64_persistent<16, 3, true>, (const void *)contract_f64_persistent<24, 1, false>,
                        (const void *)contract_f64_persistent<24, 3, false>, (const void *)contract_f64_persistent<24, 3, true>,
                        (const void *)contract_f64_persistent<32, 1, false>, (const void *)contract_f64_persistent<32, 3, false>,
                        (const void *)contract_f64_persistent<32, 3, true>,
                        (const void *)contract_f64_wide_kernel<1, false>, (const void *)contract_f64_wide_kernel<3, false>,
                        (const void *)contract_f64_wide_kernel<3, true>, (const void *)contract_f64_wide_persistent<1, false>,
                        (const void *)contract_f64_wide_persistent<3, false>, (const void *)contract_f64_wide_persistent<3, true>};
    for (const void *k : ks) PUFE_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds));
    return hipSuccess;
}

size_t contract_wide_lds_bytes(int rows, int nfun, int nimg, int nleaf, int n3) {
    return ContractLds<kWideQ>::bytes(rows, nfun, nimg, nleaf, n3) + sizeof(int) * 4 * kWideWaves;
}

hipError_t launch_contract_wide(int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items,
                                const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                                const uint32_t *leaves, const double *V, double *partial, size_t lds, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
#define PUFE_WIDE(LL, TT)                                                                                           \
    hipLaunchKernelGGL((contract_f64_wide_kernel<LL, TT>), dim3(n_items), dim3(64 * kWideWaves), lds, st, kp, items, \
                       elems, groups, img, edof, leaves, V, partial)
    if (gen) PUFE_WIDE(3, true);
    else if (lmax <= 1) PUFE_WIDE(1, false);
    else PUFE_WIDE(3, false);
#undef PUFE_WIDE
    return hipGetLastError();
}

hipError_t launch_contract_wide_persistent(int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items,
                                           int *counter, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, counter);
    PUFE_HIP(hipGetLastError());
    if (n_items == 0) return hipSuccess;
#define PUFE_WIDE_P(LL, TT)                                                                                           \
    hipLaunchKernelGGL((contract_f64_wide_persistent<LL, TT>), dim3(grid), dim3(64 * kWideWaves), lds, st, ctxs, items, \
                       n_items, counter)
    if (gen) PUFE_WIDE_P(3, true);
    else if (lmax <= 1) PUFE_WIDE_P(1, false);
    else PUFE_WIDE_P(3, false);
#undef PUFE_WIDE_P
    return hipGetLastError();
}

int persistent_blocks_per_cu(size_t lds) {
    int per = (int)((size_t)160 * 1024 / (lds > 0 ? lds : 1));   // the CU's LDS
    if (per > 2) per = 2;  // 256 VGPRs per lane: one 4-wave group per SIMD set, two if LDS allows
    return per < 1 ? 1 : per;
}

hipError_t launch_contract_persistent(int q, int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items,
                                      int *counter, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, counter);
    PUFE_HIP(hipGetLastError());
    if (n_items == 0) return hipSuccess;
#define PUFE_PERSIST(QQ, LL, TT)                                                                                     \
    hipLaunchKernelGGL((contract_f64_persistent<QQ, LL, TT>), dim3(grid), dim3(kContractThreads), lds, st, ctxs, items, \
                       n_items, counter)
#define PUFE_PERSIST_Q(QQ)                          \
    do {                                            \
        if (gen) PUFE_PERSIST(QQ, 3, true);         \
        else if (lmax <= 1) PUFE_PERSIST(QQ, 1, false); \
        else PUFE_PERSIST(QQ, 3, false);            \
    } while (0)
    if (q == 32) PUFE_PERSIST_Q(32);
    else if (q == 24) PUFE_PERSIST_Q(24);
    else PUFE_PERSIST_Q(16);
#undef PUFE_PERSIST_Q
#undef PUFE_PERSIST
    return hipGetLastError();
}

hipError_t launch_chunk_reduce(const ElemDev *elems, const int2 *list, int n, double *partial, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_reduce_kernel, dim3(n), dim3(256), 0, st, elems, list, partial);
    return hipGetLastError();
}

hipError_t launch_chunk_reduce_batch(const CtxDev *ctxs, const int4 *list, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_reduce_batch_kernel, dim3(n), dim3(256), 0, st, ctxs, list);
    return hipGetLastError();
}

hipError_t launch_phase_table(const KPoints &kps, double2 *z, hipStream_t st) {
    hipLaunchKernelGGL(phase_table_kernel, dim3((kps.nk * 27 + 127) / 128), dim3(128), 0, st, kps, z);
    return hipGetLastError();
}

hipError_t launch_scatter_batch(const CtxDev *ctxs, const int4 *list, int n, const double2 *z, int nk,
                                int out_dtype, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_batch_kernel, dim3(n), dim3(256), 0, st, ctxs, list, z, nk, out_dtype);
    return hipGetLastError();
}

hipError_t launch_prepare_outputs(void *H, void *S, int64_t bytes, const KPoints &kps, double2 *z, hipStream_t st) {
    if (bytes % 8 != 0) return hipErrorInvalidValue;
    const int64_t nw = bytes / 8;
    int64_t blocks = (nw + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(prepare_outputs_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (double *)H, (double *)S, nw,
                       kps, z);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, int64_t n, bool f32, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (f32)
        hipLaunchKernelGGL(fill_zero_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (float *)p, n);
    else
        hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (double *)p, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const KParams &kp, const ElemDev *elems, const int2 *list, int n, const int32_t *edof,
                          const double *partial, const double2 *z, int nk, int out_dtype, void *H, void *S,
                          int64_t nnz, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3(n), dim3(256), 0, st, kp, elems, list, edof, partial, z, nk, out_dtype, H,
                       S, nnz);
    return hipGetLastError();
}

hipError_t launch_elem_matrices(const ElemDev *elems, int64_t e, const double *partial, double *He, double *Se,
                                int ld, hipStream_t st) {
    hipLaunchKernelGGL(elem_matrices_kernel, dim3(16), dim3(256), 0, st, elems, e, partial, He, Se, ld);
    return hipGetLastError();
}

hipError_t launch_bsr_to_dense(int64_t nnzb, const int32_t *brow, const int32_t *bcol, const int64_t *bval_off,
                               const int64_t *dof_off, const void *src, int dtype, int64_t n, double *dense,
                               hipStream_t st) {
    int64_t blocks = nnzb < 65535 ? nnzb : 65535;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(bsr_to_dense_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nnzb, brow, bcol, bval_off,
                       dof_off, src, dtype, n, dense);
    return hipGetLastError();
}

}  // namespace pufe
