// Error-driven adaptive quadrature (section "Adaptive quadrature"), level
// by level on the device.
//
// Every open octree cell integrates Psi^2 and |grad Psi|^2 of each enrichment
// function still in its mask with the base n^3 Gauss rule and the reference
// n_ref^3 rule; a function fails when either absolute difference exceeds the
// tolerance.  A cell with failures below the maximum level is replaced by its
// 8 children, which inherit only the failing functions; otherwise it becomes a
// leaf.  The cell list is kept element-major and depth first: a split cell is
// replaced in place by its children c = c1 + 2 c2 + 4 c3, so the final list
// is the leaf order of the rule.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aq_error.hpp"
#include "enrich.hpp"
#include "tables.hpp"

namespace pufe {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int L>
__device__ __forceinline__ void cell_group_test(const KParams &kp, const GroupDev &G, const double *img,
                                                const double *org, uint32_t code, double tol, uint64_t mask,
                                                uint64_t *fail, double *red) {
    constexpr int NM = 2 * L + 1;
    const int lev = (int)(code >> 27);
    const int cc[3] = {(int)(code & 511u), (int)((code >> 9) & 511u), (int)((code >> 18) & 511u)};
    const double h = 1.0 / (double)(1 << lev);
    const int nb = kp.n3, nr = kp.nref * kp.nref * kp.nref;
    double acc[NM][4];
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m][0] = acc[m][1] = acc[m][2] = acc[m][3] = 0.0;
    for (int p = threadIdx.x; p < nb + nr; p += blockDim.x) {
        const bool base = p < nb;
        const int j = base ? p : p - nb;
        const int n = base ? kp.n : kp.nref;
        const double *gx = base ? kp.gx : kp.rx, *gw = base ? kp.gw : kp.rw;
        const int k[3] = {j % n, (j / n) % n, j / (n * n)};
        double xi[3], w = h * h * h * kp.jac;
        for (int d = 0; d < 3; ++d) {
            xi[d] = -1.0 + (2.0 * cc[d] + 1.0 + gx[k[d]]) * h;
            w *= gw[k[d]];
        }
        double x[3];
        for (int c = 0; c < 3; ++c)
            x[c] = org[c] + 0.5 * (xi[0] + 1.0) * kp.E[c] + 0.5 * (xi[1] + 1.0) * kp.E[3 + c] +
                   0.5 * (xi[2] + 1.0) * kp.E[6 + c];
        double psi[NM], gp[3 * NM];
        group_eval_point<L>(G, img, kp.spl, x, psi, gp);
        const int s = base ? 0 : 1;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            acc[m][s] += w * psi[m] * psi[m];
            acc[m][2 + s] += w * (gp[3 * m] * gp[3 * m] + gp[3 * m + 1] * gp[3 * m + 1] + gp[3 * m + 2] * gp[3 * m + 2]);
        }
    }
    // deterministic reduction: within each wave, then the waves in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double v = wave_sum(acc[m][t]);
            if (lane == 0) red[(m * 4 + t) * 4 + wave] = v;
        }
    __syncthreads();
    if (threadIdx.x < NM) {
        const int m = threadIdx.x;
        double tot[4];
        for (int t = 0; t < 4; ++t) {
            tot[t] = 0.0;
            for (int wv = 0; wv < nw; ++wv) tot[t] += red[(m * 4 + t) * 4 + wv];
        }
        const int f = G.fbase + m;
        if (((mask >> f) & 1ull) && (fabs(tot[0] - tot[1]) > tol || fabs(tot[2] - tot[3]) > tol))
            atomicOr((unsigned long long *)fail, 1ull << f);
    }
    __syncthreads();
}

// One work group per cell of the current list.  count[i] = 8 if the cell
// splits, else 1; newmask[i] = failing functions.
__global__ __launch_bounds__(256) void aq_error_test_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                            const GroupDev *__restrict__ groups,
                                                            const double *__restrict__ img,
                                                            const CellDev *__restrict__ cells, int max_level,
                                                            double tol, int64_t *__restrict__ count,
                                                            uint64_t *__restrict__ newmask) {
    __shared__ double red[28 * 4];
    __shared__ unsigned long long fail;
    const CellDev cell = cells[blockIdx.x];
    const int lev = (int)(cell.code >> 27);
    if (!cell.open || lev >= max_level || cell.mask == 0ull) {
        if (threadIdx.x == 0) {
            count[blockIdx.x] = 1;
            newmask[blockIdx.x] = 0ull;
        }
        return;
    }
    if (threadIdx.x == 0) fail = 0ull;
    __syncthreads();
    const ElemDev &el = elems[cell.elem];
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};
    for (int g = 0; g < el.ngrp; ++g) {
        const GroupDev G = groups[el.grp_off + g];
        const int nm = 2 * G.l + 1;
        const uint64_t gbits = (nm >= 64 ? ~0ull : ((1ull << nm) - 1ull)) << G.fbase;
        if (!(cell.mask & gbits)) continue;
        switch (G.l) {
            case 0: cell_group_test<0>(kp, G, img, org, cell.code, tol, cell.mask, (uint64_t *)&fail, red); break;
            case 1: cell_group_test<1>(kp, G, img, org, cell.code, tol, cell.mask, (uint64_t *)&fail, red); break;
            case 2: cell_group_test<2>(kp, G, img, org, cell.code, tol, cell.mask, (uint64_t *)&fail, red); break;
            default: cell_group_test<3>(kp, G, img, org, cell.code, tol, cell.mask, (uint64_t *)&fail, red); break;
        }
    }
    if (threadIdx.x == 0) {
        count[blockIdx.x] = fail ? 8 : 1;
        newmask[blockIdx.x] = fail;
    }
}

// Next list: a kept cell is copied (closed), a split cell becomes its 8
// children carrying the failing functions.
__global__ void aq_error_expand_kernel(int64_t n, const CellDev *__restrict__ cells,
                                       const int64_t *__restrict__ off, const uint64_t *__restrict__ newmask,
                                       CellDev *__restrict__ next) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CellDev c = cells[i];
    const int64_t o = off[i];
    if (off[i + 1] - o == 1) {
        CellDev d = c;
        d.open = 0;
        next[o] = d;
        return;
    }
    const int lev = (int)(c.code >> 27);
    const int cc[3] = {(int)(c.code & 511u), (int)((c.code >> 9) & 511u), (int)((c.code >> 18) & 511u)};
    for (int ch = 0; ch < 8; ++ch) {
        CellDev d;
        d.mask = newmask[i];
        d.elem = c.elem;
        d.code = leaf_pack(lev + 1, 2 * cc[0] + (ch & 1), 2 * cc[1] + ((ch >> 1) & 1), 2 * cc[2] + ((ch >> 2) & 1));
        d.open = 1;
        d.pad = 0;
        next[o + ch] = d;
    }
}

// Root cells: one per element, testing every function the element carries.
__global__ void aq_error_init_kernel(int64_t nel, const ElemDev *__restrict__ elems, CellDev *__restrict__ cells) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nel) return;
    const int nf = elems[e].nfun;
    CellDev c;
    c.mask = nf >= 64 ? ~0ull : ((1ull << nf) - 1ull);
    c.elem = (int32_t)e;
    c.code = leaf_pack(0, 0, 0, 0);
    c.open = 1;
    c.pad = 0;
    cells[e] = c;
}

// Final list -> leaf codes, leaf elements and per-element leaf counts.
__global__ void aq_error_finish_kernel(int64_t n, const CellDev *__restrict__ cells, uint32_t *__restrict__ leaves,
                                       int32_t *__restrict__ leaf_elem, int64_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    leaves[i] = cells[i].code;
    leaf_elem[i] = cells[i].elem;
    if (i == 0 || cells[i - 1].elem != cells[i].elem) {
        int64_t j = i;
        while (j < n && cells[j].elem == cells[i].elem) ++j;
        count[cells[i].elem] = j - i;
    }
}

hipError_t launch_aq_error_init(int64_t nel, const ElemDev *elems, CellDev *cells, hipStream_t st) {
    hipLaunchKernelGGL(aq_error_init_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, st, nel, elems, cells);
    return hipGetLastError();
}

hipError_t launch_aq_error_test(const KParams &kp, const ElemDev *elems, const GroupDev *groups, const double *img,
                                const CellDev *cells, int64_t n, int max_level, double tol, int64_t *count,
                                uint64_t *newmask, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(aq_error_test_kernel, dim3((unsigned)n), dim3(256), 0, st, kp, elems, groups, img, cells,
                       max_level, tol, count, newmask);
    return hipGetLastError();
}

hipError_t launch_aq_error_expand(int64_t n, const CellDev *cells, const int64_t *off, const uint64_t *newmask,
                                  CellDev *next, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(aq_error_expand_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cells, off,
                       newmask, next);
    return hipGetLastError();
}

hipError_t launch_aq_error_finish(int64_t n, const CellDev *cells, uint32_t *leaves, int32_t *leaf_elem,
                                  int64_t *count, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(aq_error_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cells,
                       leaves, leaf_elem, count);
    return hipGetLastError();
}

}  // namespace pufe
