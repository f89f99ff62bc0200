// Split-BF16 element contraction (gfx950 v_mfma_f32_16x16x32_bf16).
//
// Every FP64 operand x is split into bf16 limbs x = x0 + x1 (+ x2) by
// round-to-nearest on the successive residuals.  A product a b is then formed
// from the limb products of the same order of magnitude:
//   BF16X3: a0 b0 + a0 b1 + a1 b0            (two limbs, three products)
//   BF16X6: ... + a1 b1 + a0 b2 + a2 b0      (three limbs, six products)
// accumulated by the MFMA in FP32 over one stage of 32 quadrature points, one
// accumulator per operand component, and added to FP64 accumulators after
// each stage.  The contraction is the one of
// eq. disceig3d restricted to an element, written symmetrically:
//   S_e = U U^T, H_e = sum_d G_d G_d^T + (V U) U^T
// with U[a][q] = sqrt(w_q) phi_a(x_q) and G_d[a][q] = sqrt(w_q / 2) d_d phi_a(x_q).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "basis.hpp"
#include "device_common.hpp"
#include "enrich.hpp"
#include "kernels.hpp"
#include "tables.hpp"

namespace pufe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));

// FP32 -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double bf16_value(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

// LDS map: limbs[j][row][comp][q] (bf16 bits, comp = grad_x, grad_y, grad_z,
// U, V U), then the FP64 enrichment functions and per-point geometry.
template <int Q>
struct SplitLds {
    static constexpr int RSB = 5 * Q * 2 + 16;  // bytes per row and limb (padded)
    static __host__ __device__ size_t bytes(int nlimb, int rows, int nfun) {
        return (size_t)nlimb * rows * RSB + sizeof(double) * ((size_t)nfun * Q * 4 + (size_t)Q * 28);
    }
};

template <int NL, int Q>
__device__ __forceinline__ void contract_split_item(
    const KParams &kp, const ItemDev &it, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial,
    unsigned char *smem_raw) {
    static_assert(Q == 32, "one S product covers 32 points");
    constexpr int RSB = SplitLds<Q>::RSB;
    const ElemDev &el = elems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun;
    const bool diag = it.I0 == it.J0;
    const int nrow = 16 * (diag ? it.nI : it.nI + it.nJ);
    unsigned char *sLimb = smem_raw;
    double *sPsi = (double *)(smem_raw + (size_t)NL * nrow * RSB);
    double *sQ = sPsi + (size_t)nfun * Q * 4;
    double *sXi = sQ, *sX = sQ + 3 * Q, *sW = sQ + 6 * Q, *sVq = sQ + 7 * Q, *sL = sQ + 8 * Q, *sD = sQ + 17 * Q;
    double *sSw = sQ + 26 * Q, *sSw2 = sQ + 27 * Q;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n3 = kp.n3;
    const int64_t q_begin = it.leaf_b * n3, q_end = it.leaf_e * n3;
    const int ti0 = it.I0, tj0 = it.J0;
    const int npairs = diag ? it.nI * (it.nI + 1) / 2 : it.nI * it.nJ;
    int pr_row[4], pr_col[4], pr_I[4], pr_J[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int pidx = wave + 4 * u;
        pr_row[u] = pr_col[u] = pr_I[u] = pr_J[u] = -1;
        if (pidx < npairs) {
            int a, b;
            if (diag) {
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
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};

    for (int64_t qb = q_begin; qb < q_end; qb += Q) {
        if (tid < Q) {
            const int64_t qg = qb + tid;
            double xi[3] = {0.0, 0.0, 0.0}, w = 0.0, vq = 0.0;
            if (qg < q_end) {
                const int64_t lf = qg / n3;
                leaf_point(kp, leaves[lf], (int)(qg - lf * n3), xi, &w);
                vq = V[qg];
            }
            for (int d = 0; d < 3; ++d) sXi[3 * tid + d] = xi[d];
            for (int c = 0; c < 3; ++c)
                sX[3 * tid + c] = org[c] + 0.5 * (xi[0] + 1.0) * kp.E[c] + 0.5 * (xi[1] + 1.0) * kp.E[3 + c] +
                                  0.5 * (xi[2] + 1.0) * kp.E[6 + c];
            sW[tid] = w;
            sVq[tid] = vq;
            sSw[tid] = sqrt(w);
            sSw2[tid] = sqrt(0.5 * w);
            for (int d = 0; d < 3; ++d) lagrange_1d(kp.p, xi[d], sL + 9 * tid + 3 * d, sD + 9 * tid + 3 * d);
        }
        __syncthreads();
        for (int idx = tid; idx < ngrp * Q; idx += 256) {
            const int g = idx / Q, q = idx - g * Q;
            const GroupDev G = groups[el.grp_off + g];
            double *o = sPsi + ((size_t)G.fbase * Q + q) * 4;
            switch (G.l) {
                case 0: group_eval<0, Q * 4, 1>(G, img, sX + 3 * q, o); break;
                case 1: group_eval<1, Q * 4, 1>(G, img, sX + 3 * q, o); break;
                case 2: group_eval<2, Q * 4, 1>(G, img, sX + 3 * q, o); break;
                default: group_eval<3, Q * 4, 1>(G, img, sX + 3 * q, o); break;
            }
        }
        __syncthreads();
        // rows: weighted operands, split into limbs
        for (int idx = tid; idx < nrow * Q; idx += 256) {
            const int r = idx / Q, q = idx - r * Q;
            const int a = (diag || r < 16 * it.nI) ? 16 * ti0 + r : 16 * tj0 + (r - 16 * it.nI);
            double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (a < nloc && sW[q] != 0.0) {
                double val, g[3];
                if (a < nfe) {
                    const double *L = sL + 9 * q, *D = sD + 9 * q;
                    const int n1 = kp.p + 1;
                    const int a1 = a % n1, a2 = (a / n1) % n1, a3 = a / (n1 * n1);
                    const double l1 = L[a1], l2 = L[3 + a2], l3 = L[6 + a3];
                    const double dxi[3] = {D[a1] * l2 * l3, l1 * D[3 + a2] * l3, l1 * l2 * D[6 + a3]};
                    val = l1 * l2 * l3;
                    for (int c = 0; c < 3; ++c)
                        g[c] = kp.Jt[3 * c] * dxi[0] + kp.Jt[3 * c + 1] * dxi[1] + kp.Jt[3 * c + 2] * dxi[2];
                } else {
                    const int pk = edof[el.edof_off + (a - nfe)];
                    const int c = pk & 7, f = (pk >> 3) & 255;
                    double m[3], dm[3];
                    for (int d = 0; d < 3; ++d) {
                        const double t = sXi[3 * q + d];
                        const int bit = (c >> d) & 1;
                        m[d] = bit ? 0.5 * (1.0 + t) : 0.5 * (1.0 - t);
                        dm[d] = bit ? 0.5 : -0.5;
                    }
                    const double M = m[0] * m[1] * m[2];
                    const double dM[3] = {dm[0] * m[1] * m[2], m[0] * dm[1] * m[2], m[0] * m[1] * dm[2]};
                    const double *ps = sPsi + ((size_t)f * Q + q) * 4;
                    for (int cc = 0; cc < 3; ++cc) {
                        const double gM = kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2];
                        g[cc] = gM * ps[0] + M * ps[1 + cc];
                    }
                    val = M * ps[0];
                }
                const double s2 = sSw2[q], s1 = sSw[q];
                v[0] = s2 * g[0];
                v[1] = s2 * g[1];
                v[2] = s2 * g[2];
                v[3] = s1 * val;
                v[4] = sVq[q] * v[3];
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                double x = v[c];
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    const uint16_t h = bf16_bits((float)x);
                    *(uint16_t *)(sLimb + ((size_t)j * nrow + r) * RSB + (size_t)(c * Q + q) * 2) = h;
                    x -= bf16_value(h);
                }
            }
        }
        __syncthreads();
        // MFMA over limb products; lane = i + 16 grp holds the 8 consecutive
        // points 8 grp .. 8 grp + 7 of one component.  Every component (the
        // three gradient components and V U against U for H, U against U for
        // S) gets its own FP32 accumulator over the stage's 32 points, added
        // to the FP64 accumulators afterwards: terms of one magnitude class
        // share an FP32 sum, so the MFMA's internal FP32 rounding stays at the
        // scale of that component rather than of the largest one.
        const int r16 = lane & 15, grp = lane >> 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (pr_row[u] < 0) continue;
            const unsigned char *rowA = sLimb + (size_t)(pr_row[u] + r16) * RSB;
            const unsigned char *rowB = sLimb + (size_t)(pr_col[u] + r16) * RSB;
            const size_t LS = (size_t)nrow * RSB;  // limb stride
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
                f32x4 h = {0.f, 0.f, 0.f, 0.f};
                if (NL == 3) {
                    h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], h, 0, 0, 0);
                    h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], h, 0, 0, 0);
                    h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], h, 0, 0, 0);
                }
                h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], h, 0, 0, 0);
                h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], h, 0, 0, 0);
                h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], h, 0, 0, 0);
                if (c < 4) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) accH[u][r] += (double)h[r];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) accS[u][r] += (double)h[r];
                }
            }
        }
        __syncthreads();
    }
    const int T = (nloc + 15) / 16;
    const int64_t P = (int64_t)T * (T + 1) / 2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (pr_row[u] < 0) continue;
        const int64_t pidx = (int64_t)pr_J[u] * (pr_J[u] + 1) / 2 + pr_I[u];
        double *dst = partial + (el.part_base + (int64_t)it.chunk * P + pidx) * 512;
        const int j = lane & 15, i0 = 4 * (lane >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dst[(i0 + r) * 16 + j] = accH[u][r];
            dst[256 + (i0 + r) * 16 + j] = accS[u][r];
        }
    }
}

template <int NL, int Q>
__global__ __launch_bounds__(256) void contract_split_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, double *__restrict__ partial) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const ItemDev it = items[blockIdx.x];
    contract_split_item<NL, Q>(kp, it, elems, groups, img, edof, leaves, V, partial, smem_raw);
}

// Persistent queue form (see contract_f64_persistent).
template <int NL, int Q>
__global__ __launch_bounds__(256) void contract_split_persistent(const CtxDev *__restrict__ ctxs,
                                                                 const ItemDev *__restrict__ items, int n_items,
                                                                 int *__restrict__ counter) {
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
        contract_split_item<NL, Q>(c.kp, it, c.elems, c.groups, c.img, c.edof, c.leaves, c.V, c.partial, smem_raw);
    }
}

__global__ void reset_counter_split_kernel(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

hipError_t launch_split_persistent(int nlimb, const CtxDev *ctxs, const ItemDev *items, int n_items, int *counter,
                                   int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_split_kernel, dim3(1), dim3(64), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n_items == 0) return hipSuccess;
    if (nlimb == 2)
        hipLaunchKernelGGL((contract_split_persistent<2, kSplitQ>), dim3(grid), dim3(256), lds, st, ctxs, items,
                           n_items, counter);
    else
        hipLaunchKernelGGL((contract_split_persistent<3, kSplitQ>), dim3(grid), dim3(256), lds, st, ctxs, items,
                           n_items, counter);
    return hipGetLastError();
}

hipError_t init_split_attributes() {
    const void *ks[4] = {(const void *)contract_split_kernel<2, kSplitQ>, (const void *)contract_split_kernel<3, kSplitQ>,
                         (const void *)contract_split_persistent<2, kSplitQ>,
                         (const void *)contract_split_persistent<3, kSplitQ>};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t split_lds_bytes(int nlimb, int rows, int nfun) { return SplitLds<kSplitQ>::bytes(nlimb, rows, nfun); }

hipError_t launch_contract_split(int nlimb, const KParams &kp, int n_items, const ItemDev *items, const ElemDev *elems,
                                 const GroupDev *groups, const double *img, const int32_t *edof,
                                 const uint32_t *leaves, const double *V, double *partial, size_t lds,
                                 hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (nlimb == 2)
        hipLaunchKernelGGL((contract_split_kernel<2, kSplitQ>), dim3(n_items), dim3(256), lds, st, kp, items, elems,
                           groups, img, edof, leaves, V, partial);
    else
        hipLaunchKernelGGL((contract_split_kernel<3, kSplitQ>), dim3(n_items), dim3(256), lds, st, kp, items, elems,
                           groups, img, edof, leaves, V, partial);
    return hipGetLastError();
}

}  // namespace pufe
