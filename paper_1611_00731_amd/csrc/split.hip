// Split-BF16 element contraction (gfx950 v_mfma_f32_16x16x32_bf16).
//
// Every FP64 operand x is split into bf16 limbs x = x0 + x1 (+ x2) by
// round-to-nearest on the successive residuals.  A product a b is then formed
// from the limb products of the same order of magnitude:
//   BF16X3: a0 b0 + a0 b1 + a1 b0            (two limbs, three products)
//   BF16X6: ... + a1 b1 + a0 b2 + a2 b0      (three limbs, six products)
// One MFMA sums 32 points of one operand component; every component (the
// three gradient components and V u for H, u for S) has its own FP32
// accumulator per 32-point stage, added to FP64 accumulators after each
// stage, so the MFMA's FP32 rounding stays at the scale of that component.
// The contraction is the one of eq. disceig3d restricted to an element,
// written symmetrically:
//   S_e = U U^T, H_e = sum_d G_d G_d^T + (V U) U^T
// with U[a][q] = sqrt(w_q) phi_a(x_q) and G_d[a][q] = sqrt(w_q / 2) d_d phi_a(x_q).
// The per-point geometry, the enrichment functions and the FP64 basis rows
// are built as in the FP64 kernel (stage.hpp) and split into limbs in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "limbs.hpp"
#include "stage.hpp"
#include "tables.hpp"

namespace pufe {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kSplitThreads = 256;

// LDS map (per work item):
//   sLimb[j][row][5][Q]  bf16 limb j of the weighted operands sqrt(w/2) d_x phi,
//                        sqrt(w/2) d_y phi, sqrt(w/2) d_z phi, sqrt(w) phi,
//                        V sqrt(w) phi (row stride RSB bytes)
//   sV[Q], sPsi[f][4][Q], sGeo[GEO][Q], sImg, sGx, sGs   (FP64)
//   sG, sEd, sLeaf, sPt, sRow
template <int Q>
struct SplitLds {
    static constexpr int RSB = 5 * Q * 2 + 16;  // bytes per row and limb: 16-byte rows, 20-word bank offset
    static constexpr int GEO = 40;
    static __host__ __device__ size_t bytes(int nlimb, int rows, int nfun, int nimg, int nleaf, int n3) {
        return (size_t)nlimb * rows * RSB +
               sizeof(double) * ((size_t)Q + (size_t)nfun * Q * 4 + (size_t)Q * GEO + (size_t)nimg * 3 +
                                 2 * kMaxGauss) +
               sizeof(GroupDev) * kMaxGroups + sizeof(int32_t) * kMaxNloc +
               sizeof(uint32_t) * ((size_t)nleaf + n3 + rows) + 64;
    }
};

template <int NL, int Q, int LMAX, bool GEN>
__device__ __forceinline__ void contract_split_item(
    const KParams &kpg, const ItemDev &it, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial,
    unsigned char *smem_raw) {
    static_assert(Q == 32, "one MFMA covers the 32 points of a stage");
    constexpr int RSB = SplitLds<Q>::RSB;
    constexpr int GEO = SplitLds<Q>::GEO;
    constexpr int NT = kSplitThreads;
    const KLocal kp = load_klocal(kpg);
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
    unsigned char *sLimb = smem_raw;                                          // [NL][nrow][RSB]
    double *sV = (double *)(smem_raw + (size_t)NL * nrow * RSB);              // [Q]
    double *sPsi = sV + Q;                                                    // [nfun][4][Q]
    double *sGeo = sPsi + (size_t)nfun * Q * 4;                               // [GEO][Q]
    double *sImg = sGeo + (size_t)Q * GEO;
    double *sGx = sImg + 3 * (size_t)nimg, *sGs = sGx + kMaxGauss;   // square roots of the 1D Gauss weights
    GroupDev *sG = (GroupDev *)(sGs + kMaxGauss);
    int32_t *sEd = (int32_t *)(sG + kMaxGroups);
    uint32_t *sLeaf = (uint32_t *)(sEd + kMaxNloc);
    uint32_t *sPt = sLeaf + (it.leaf_e - it.leaf_b);
    int *sRow = (int *)(sPt + n3);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q_begin = it.leaf_b * (int64_t)n3, q_end = it.leaf_e * (int64_t)n3;
    const uint32_t nli = (uint32_t)(q_end - q_begin);
    const int ti0 = it.I0, tj0 = it.J0;
    for (int k = tid; k < nloc - nfe; k += NT) sEd[k] = gEdof[el.edof_off + k];
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
    for (int k = tid; k < 3 * nimg; k += NT) sImg[k] = gImg[3 * (size_t)img0 + k];
    for (int64_t k = tid; k < it.leaf_e - it.leaf_b; k += NT) sLeaf[k] = gLeaves[it.leaf_b + k];
    for (uint32_t j = tid; j < n3; j += NT) sPt[j] = (j % n) | (((j / n) % n) << 8) | ((j / (n * n)) << 16);
    for (int r = tid; r < nrow; r += NT) {
        const int a = (diag || r < 16 * it.nI) ? 16 * ti0 + r : 16 * tj0 + (r - 16 * it.nI);
        sRow[r] = a < nloc ? a : -1;
    }
    if (tid < kp.n) {
        sGx[tid] = kpg.gx[tid];
        sGs[tid] = sqrt(kpg.gw[tid]);
    }
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};

    // tile pairs of this item, round-robin over the four waves
    const int npairs = diag ? it.nI * (it.nI + 1) / 2 : it.nI * it.nJ;
    int pr_row[4], pr_col[4], pr_I[4], pr_J[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int pidx = wave + 4 * u;
        pr_row[u] = pr_col[u] = pr_I[u] = pr_J[u] = -1;
        if (pidx < npairs) {
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
    double4_t accH[4], accS[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        accH[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
        accS[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
    }
    // the last Q threads build the geometry; V is read one stage ahead
    const int gq = tid - (NT - Q);
    double v = (gq >= 0 && (uint32_t)gq < nli) ? gV[q_begin + gq] : 0.0;
    __syncthreads();

    // phase 1 of the stage starting at lbx: enrichment functions (eq. Psi,
    // f(R) = 1), geometry and V
    auto phase1 = [&](uint32_t lbx) {
        if (gq >= 0) {
            const double vn = (lbx + Q + gq < nli) ? gV[q_begin + lbx + Q + gq] : 0.0;
            double xi[3], sw;
            item_point(kp, sLeaf, sPt, sGx, sGs, lbx + gq, nli, n3, xi, &sw);
            point_geometry<Q>(kp, org, xi, sw, sGeo + gq);
            sV[gq] = v;
            v = vn;
        }
        for (int idx = tid; idx < ngrp * Q; idx += NT) {
            const int g = idx / Q, q = idx - g * Q;
            const GroupDev &G = sG[g];
            double xi[3], sw, x[3];
            item_point(kp, sLeaf, sPt, sGx, sGs, lbx + q, nli, n3, xi, &sw);
            point_position(kp, org, xi, x);
            group_eval_upto<LMAX, Q, 4 * Q, GEN>(G, sImg, kp.spl, wimg, x, sPsi + (size_t)G.fbase * 4 * Q + q);
        }
    };
    if (nli > 0) phase1(0);
    __syncthreads();
    for (uint32_t lb = 0; lb < nli; lb += Q) {
        // ---- phase 2: weighted rows at two adjacent points per thread, split
        // into limbs and stored as bf16 pairs
        for (int idx = tid; idx < nrow * (Q / 2); idx += NT) {
            const int r = idx / (Q / 2), q0 = 2 * (idx - r * (Q / 2));
            const int a = sRow[r];
            double comp[2][5];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int q = q0 + t;
                const double *g = sGeo + q;
                double val, gx[3];
                local_row<Q, GEN>(kp, g, sPsi + q, sEd, a, nfe, &val, gx);
                const double s2 = g[G_SW2 * Q], u = g[G_SW * Q] * val;
                comp[t][0] = s2 * gx[0];
                comp[t][1] = s2 * gx[1];
                comp[t][2] = s2 * gx[2];
                comp[t][3] = u;
                comp[t][4] = sV[q] * u;
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                uint32_t hp[NL];
                split_limbs2<NL>(comp[0][c], comp[1][c], hp);
#pragma unroll
                for (int j = 0; j < NL; ++j)
                    *(uint32_t *)(sLimb + ((size_t)j * nrow + r) * RSB + (size_t)(c * Q + q0) * 2) = hp[j];
            }
        }
        __syncthreads();
        // ---- phase 3 of this stage and phase 1 of the next share one barrier
        // interval (phase 3 reads only the limbs); MFMAs over limb products; lane = i + 16 grp holds the 8
        // consecutive points 8 grp .. 8 grp + 7 of one component
        {
            const int r16 = lane & 15, grp = lane >> 4;
            const size_t LS = (size_t)nrow * RSB;  // limb stride
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (pr_row[u] < 0) continue;
                const unsigned char *rowA = sLimb + (size_t)(pr_row[u] + r16) * RSB;
                const unsigned char *rowB = sLimb + (size_t)(pr_col[u] + r16) * RSB;
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    // c = 0..2: gradient components (H); 3: V U x U (H); 4: U x U (S)
                    const int ca = c < 3 ? c : (c == 3 ? 4 : 3), cb = c < 3 ? c : 3;
                    const size_t offA = (size_t)(ca * Q + 8 * grp) * 2, offB = (size_t)(cb * Q + 8 * grp) * 2;
                    bf16x8 A[NL], B[NL];
#pragma unroll
                    for (int j = 0; j < NL; ++j) {
                        A[j] = *(const bf16x8 *)(rowA + j * LS + offA);
                        B[j] = *(const bf16x8 *)(rowB + j * LS + offB);
                    }
                    const f32x4 h = mfma_limbs<NL>(A, B, (f32x4){0.f, 0.f, 0.f, 0.f});
                    if (c < 4) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) accH[u][r] += (double)h[r];
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) accS[u][r] += (double)h[r];
                    }
                }
            }
        }
        if (lb + Q < nli) phase1(lb + Q);
        __syncthreads();
    }
    // ---- partial tiles, row-major 16x16.  bf16 16x16x32 accumulator layout:
    // register r of lane l holds D[4 (l / 16) + r][l % 16].
    const int T = (nloc + 15) / 16;
    const int64_t P = (int64_t)T * (T + 1) / 2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (pr_row[u] < 0) continue;
        const int64_t pidx = (int64_t)pr_J[u] * (pr_J[u] + 1) / 2 + pr_I[u];
        PUFE_GLOBAL double *dst = gPartial + (el.part_base + (int64_t)it.chunk * P + pidx) * 512;
        const int j = lane & 15, i0 = 4 * (lane >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dst[(i0 + r) * 16 + j] = accH[u][r];
            dst[256 + (i0 + r) * 16 + j] = accS[u][r];
        }
    }
}

template <int NL, int Q, int LMAX, bool GEN>
__global__ __launch_bounds__(kSplitThreads) void contract_split_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const ItemDev it = items[blockIdx.x];
    contract_split_item<NL, Q, LMAX, GEN>(kp, it, elems, groups, img, edof, leaves, V, partial, smem_raw);
}

// Persistent queue form (see contract_f64_persistent).
template <int NL, int Q, int LMAX, bool GEN>
__global__ __launch_bounds__(kSplitThreads) void contract_split_persistent(const CtxDev *__restrict__ ctxs,
                                                                           const ItemDev *__restrict__ items,
                                                                           int n_items, int *__restrict__ counter) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= n_items) break;
        const ItemDev it = items[idx];
        const CtxDev &c = ctxs[it.ctx];
        contract_split_item<NL, Q, LMAX, GEN>(c.kp, it, c.elems, c.groups, c.img, c.edof, c.leaves, c.V, c.partial,
                                              smem_raw);
    }
}

__global__ void reset_counter_split_kernel(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Variants: analytic radials and Lagrange elements for l <= 1 and l <= 3, and
// the general variant (tabulated radials, serendipity elements; l <= 3).
#define PUFE_SPLIT_DISPATCH(KERNEL, NLIMB, LM, GEN, ...)                                      \
    do {                                                                                     \
        if (NLIMB == 2) {                                                                    \
            if (GEN) hipLaunchKernelGGL((KERNEL<2, kSplitQ, 3, true>), __VA_ARGS__);          \
            else if (LM <= 1) hipLaunchKernelGGL((KERNEL<2, kSplitQ, 1, false>), __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<2, kSplitQ, 3, false>), __VA_ARGS__);             \
        } else {                                                                             \
            if (GEN) hipLaunchKernelGGL((KERNEL<3, kSplitQ, 3, true>), __VA_ARGS__);          \
            else if (LM <= 1) hipLaunchKernelGGL((KERNEL<3, kSplitQ, 1, false>), __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<3, kSplitQ, 3, false>), __VA_ARGS__);             \
        }                                                                                    \
    } while (0)

hipError_t launch_split_persistent(int nlimb, int lmax, bool gen, const CtxDev *ctxs, const ItemDev *items, int n_items,
                                   int *counter, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_split_kernel, dim3(1), dim3(64), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n_items == 0) return hipSuccess;
    PUFE_SPLIT_DISPATCH(contract_split_persistent, nlimb, lmax, gen, dim3(grid), dim3(kSplitThreads), lds, st, ctxs,
                        items, n_items, counter);
    return hipGetLastError();
}

hipError_t init_split_attributes() {
    const void *ks[] = {(const void *)contract_split_kernel<2, kSplitQ, 1, false>,
                        (const void *)contract_split_kernel<2, kSplitQ, 3, false>,
                        (const void *)contract_split_kernel<2, kSplitQ, 3, true>,
                        (const void *)contract_split_kernel<3, kSplitQ, 1, false>,
                        (const void *)contract_split_kernel<3, kSplitQ, 3, false>,
                        (const void *)contract_split_kernel<3, kSplitQ, 3, true>,
                        (const void *)contract_split_persistent<2, kSplitQ, 1, false>,
                        (const void *)contract_split_persistent<2, kSplitQ, 3, false>,
                        (const void *)contract_split_persistent<2, kSplitQ, 3, true>,
                        (const void *)contract_split_persistent<3, kSplitQ, 1, false>,
                        (const void *)contract_split_persistent<3, kSplitQ, 3, false>,
                        (const void *)contract_split_persistent<3, kSplitQ, 3, true>};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t split_lds_bytes(int nlimb, int rows, int nfun, int nimg, int nleaf, int n3) {
    return SplitLds<kSplitQ>::bytes(nlimb, rows, nfun, nimg, nleaf, n3);
}

hipError_t launch_contract_split(int nlimb, int lmax, bool gen, const KParams &kp, int n_items, const ItemDev *items,
                                 const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                                 const uint32_t *leaves, const double *V, double *partial, size_t lds,
                                 hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    PUFE_SPLIT_DISPATCH(contract_split_kernel, nlimb, lmax, gen, dim3(n_items), dim3(kSplitThreads), lds, st, kp, items,
                        elems, groups, img, edof, leaves, V, partial);
    return hipGetLastError();
}

#undef PUFE_SPLIT_DISPATCH

}  // namespace pufe
