// Separable nonlocal term of the PUFE Hamiltonian (eq. disceig3d) on gfx950:
//   H_ij += sum_J h_J f_J^i conj(f_J^j),
//   f_J^i = int phi_i^* sum_n exp(i k . a_n) v_J(x - tau - a_n) dx.
// Formulation with Bloch phases on the FE and PU functions (phi_i = p_a N_a
// on an element) and projector images n:
//   f_J^i = sum_{(e, a) -> i} conj(p_a) sum_{images n of J reaching e}
//           exp(2 pi i kappa . n) F_e[a][col(J, n)],
//   F_e[a][c] = sum_q w_q N_a(x_q) v_c(x_q)          (real, k-independent)
// F_e is a contraction of the element's basis values with its projector
// values over the quadrature points, on FP64 MFMA (nl_f_kernel); with the
// Bloch-periodic enrichment the element's rows are its real rows and the
// imaginary parts of its enriched functions (images weighted per k-point), so
// F_e is per k-point and the gather takes conj(phi) = real - i imaginary, with
// the boundary phase on the classical FE rows only; the
// phases and the sum over the elements of a DOF are a gather per (J, DOF)
// (nl_gather_kernel), and the low-rank update runs per BSR block that a
// projector image couples (nl_update_kernel).  No atomics; fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "basis.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "nonlocal.hpp"
#include "stage.hpp"
#include "tables.hpp"

namespace pufe {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kNlQ = 16;        // points per stage
constexpr int kNlQU = kNlQ + 1; // row stride (doubles) of the value and projector tables: offset banks
constexpr int kNlThreads = 256;

// LDS map (per work item):
//   sU[npad][QU]     sqrt(w) N_a at the stage points (rows past nloc zero)
//   sPv[ncp][QU]     sqrt(w) v_c at the stage points (columns past ncol zero)
//   sPsi[f][4 Q]     enrichment functions (value, gradient)
//   sGeo[GEO][Q]     per-point geometry
//   sImg, sG, sPG, sEd, sCS, sLeaf, sPt, sGx, sGs
struct NlLds {
    static __host__ __device__ size_t bytes(int npad, int ncp, int nfun, int nimg, int nleaf, int n3) {
        return sizeof(double) * ((size_t)npad * kNlQU + (size_t)ncp * kNlQU + (size_t)nfun * 4 * kNlQ +
                                 (size_t)40 * kNlQ + (size_t)nimg * 3 + 2 * kMaxGauss) +
               sizeof(GroupDev) * kMaxGroups + sizeof(PGroupDev) * kMaxPGroups + sizeof(int32_t) * (kMaxNloc + 16) +
               sizeof(uint32_t) * ((size_t)nleaf + n3) + 64;
    }
};

// Projector coefficients of one element over one range of leaves, for the
// item's row tiles R0 .. R0 + nR - 1 against every column tile: FP64 MFMAs
// (v_mfma_f64_16x16x4f64, k = 4 points per instruction).
template <int LMAX>
__global__ __launch_bounds__(kNlThreads) void nl_f_kernel(
    const KParams kpg, const NlItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const PGroupDev *__restrict__ pgroups, double *__restrict__ Fp) {
    constexpr int Q = kNlQ, QU = kNlQU, NT = kNlThreads;
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const NlItemDev it = items[blockIdx.x];
    const KLocal kp = load_klocal(kpg);
    const ElemDev &el = elems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun, npg = el.npg, ncol = el.ncol;
    const int T = (nloc + 15) / 16, npad = 16 * T, TC = (ncol + 15) / 16, ncp = 16 * TC;
    const int img0 = ngrp > 0 ? groups[el.grp_off].img_off : 0;
    const int nimg = ngrp > 0 ? groups[el.grp_off + ngrp - 1].img_off + groups[el.grp_off + ngrp - 1].nimg - img0 : 0;
    const uint32_t n3 = (uint32_t)kp.n3, n = (uint32_t)kp.n;
    double *sU = smem;
    double *sPv = sU + (size_t)npad * QU;
    double *sPsi = sPv + (size_t)ncp * QU;
    double *sGeo = sPsi + (size_t)nfun * 4 * Q;
    double *sImg = sGeo + 40 * Q;
    double *sGx = sImg + 3 * (size_t)nimg, *sGs = sGx + kMaxGauss;
    GroupDev *sG = (GroupDev *)(sGs + kMaxGauss);
    PGroupDev *sPG = (PGroupDev *)(sG + kMaxGroups);
    int32_t *sEd = (int32_t *)(sPG + kMaxPGroups);
    int *sCS = sEd + kMaxNloc;
    uint32_t *sLeaf = (uint32_t *)(sCS + 16);
    uint32_t *sPt = sLeaf + (it.leaf_e - it.leaf_b);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nli = (uint32_t)((it.leaf_e - it.leaf_b) * n3);
    for (int k = tid; k < nloc - nfe; k += NT) sEd[k] = edof[el.edof_off + k];
    corner_starts((const PUFE_GLOBAL int32_t *)(edof + el.edof_off), nloc - nfe, sCS, tid, NT);
    for (int g = tid; g < ngrp; g += NT) {
        GroupDev G = groups[el.grp_off + g];
        G.img_off -= img0;
        sG[g] = G;
    }
    for (int g = tid; g < npg; g += NT) sPG[g] = pgroups[el.pg_off + g];
    for (int k = tid; k < 3 * nimg; k += NT) sImg[k] = img[3 * (size_t)img0 + k];
    for (int64_t k = tid; k < it.leaf_e - it.leaf_b; k += NT) sLeaf[k] = leaves[it.leaf_b + k];
    for (uint32_t j = tid; j < n3; j += NT) sPt[j] = (j % n) | (((j / n) % n) << 8) | ((j / (n * n)) << 16);
    // padding rows and columns stay zero
    for (int k = tid; k < (npad - nloc) * QU; k += NT) sU[(size_t)nloc * QU + k] = 0.0;
    for (int k = tid; k < (ncp - ncol) * QU; k += NT) sPv[(size_t)ncol * QU + k] = 0.0;
    if (tid < kp.n) {
        sGx[tid] = kpg.gx[tid];
        sGs[tid] = sqrt(kpg.gw[tid]);
    }
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};
    // tile pairs (row tile, column tile) of the item, round-robin over waves
    const int npairs = it.nR * TC;
    int pr_row[4], pr_col[4];
    double4_t acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int pidx = wave + 4 * u;
        pr_row[u] = pidx < npairs ? 16 * (it.R0 + pidx / TC) : -1;
        pr_col[u] = pidx < npairs ? 16 * (pidx % TC) : -1;
        acc[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
    }
    const int nfu = fe_units(kp.p);
    const int r16 = lane & 15, k4 = lane >> 4;
    __syncthreads();
    for (uint32_t lb = 0; lb < nli; lb += Q) {
        // ---- phase 1: geometry, enrichment functions, projector values
        const int gq = tid - (NT - Q);
        if (gq >= 0) {
            double xi[3], sw;
            item_point(kp, sLeaf, sPt, sGx, sGs, lb + gq, nli, n3, xi, &sw);
            point_geometry<Q>(kp, org, xi, sw, sGeo + gq);
        }
        for (int idx = tid; idx < ngrp * Q; idx += NT) {
            const int g = idx / Q, q = idx - g * Q;
            const GroupDev &G = sG[g];
            double xi[3], sw, x[3];
            item_point(kp, sLeaf, sPt, sGx, sGs, lb + q, nli, n3, xi, &sw);
            point_position(kp, org, xi, x);
            group_eval_upto<LMAX, Q>(G, sImg, kp.spl, kp.wimg ? kp.wimg + img0 : nullptr, x,
                                     sPsi + (size_t)G.fbase * 4 * Q + q);
        }
        for (int idx = tid; idx < npg * Q; idx += NT) {
            const int g = idx / Q, q = idx - g * Q;
            const PGroupDev &G = sPG[g];
            double xi[3], sw, x[3];
            item_point(kp, sLeaf, sPt, sGx, sGs, lb + q, nli, n3, xi, &sw);
            point_position(kp, org, xi, x);
            const double rx = x[0] - G.c[0], ry = x[1] - G.c[1], rz = x[2] - G.c[2];
            const double s = rx * rx + ry * ry + rz * rz, rc2 = G.rc * G.rc;
            double rad = 0.0;
            if (s < rc2) {
                const double c = 1.0 - s / rc2;
                rad = sw * exp(-G.a * s) * c * c * c;
            }
            double S[7], dS[21];
            solid_harmonics(G.l, rx, ry, rz, S, dS);
            for (int m = 0; m <= 2 * G.l; ++m) sPv[(size_t)(G.col0 + m) * QU + q] = rad * S[m];
        }
        __syncthreads();
        // ---- phase 2: sqrt(w) N_a of every local function (grouped units)
        for (int idx = tid; idx < (nfu + 8) * Q; idx += NT) {
            const int u = idx / Q, q = idx - u * Q;
            auto put = [&](int a, double, double, double, double w) { sU[(size_t)a * QU + q] = w; };
            if (u >= nfu) {
                const int c = u - nfu;
                pu_unit<Q>(kp, sGeo + q, sPsi + q, sEd, c, sCS[c], sCS[c + 1], nfe, put);
            } else {
                fe_unit_any<Q>(kp, sGeo + q, u, put);
            }
        }
        __syncthreads();
        // ---- phase 3: F[a][c] += sum_q U[a][q] P[c][q], 4 points per MFMA
#pragma unroll
        for (int s4 = 0; s4 < Q / 4; ++s4) {
            const int o = 4 * s4 + k4;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (pr_row[u] < 0) continue;
                const double a = sU[(size_t)(pr_row[u] + r16) * QU + o];
                const double b = sPv[(size_t)(pr_col[u] + r16) * QU + o];
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // slot of this K-chunk: F[col][npad], FP64 16x16x4 accumulator layout:
    // register r of lane l is row (l / 16) + 4 r, column l % 16
    double *dst = Fp + el.pf_base + (int64_t)it.chunk * ncp * npad;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (pr_row[u] < 0) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dst[(size_t)(pr_col[u] + r16) * npad + pr_row[u] + k4 + 4 * r] = acc[u][r];
    }
}

// Sum of the K-chunk slots of one element's projector coefficients, in chunk
// order, into the first slot.
__global__ __launch_bounds__(256) void nl_reduce_kernel(const ElemDev *__restrict__ elems,
                                                        const int32_t *__restrict__ nl_elems,
                                                        double *__restrict__ Fp) {
    const ElemDev &el = elems[nl_elems[blockIdx.x]];
    const int npad = 16 * ((el.nloc + 15) / 16), ncp = 16 * ((el.ncol + 15) / 16);
    const int64_t slot = (int64_t)ncp * npad;
    double *F = Fp + el.pf_base;
    for (int64_t k = threadIdx.x; k < slot; k += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < el.pf_nchunk; ++c) s += F[c * slot + k];
        F[k] = s;
    }
}

// f_J^i for the k-points of kps: one thread per (J, DOF i); the DOF's
// (element, local function) pairs in element order, each element's
// projector images of J in group order.  bpart (Bloch-periodic enrichment,
// one k-point; null otherwise): the partner table of the enriched rows, -1
// marking an imaginary part, which enters conj(phi) with the factor -i.
__global__ __launch_bounds__(256) void nl_gather_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                        const PGroupDev *__restrict__ pgroups,
                                                        const int32_t *__restrict__ edof,
                                                        const int32_t *__restrict__ bpart,
                                                        const int64_t *__restrict__ dof_el_off,
                                                        const int2 *__restrict__ dof_el,
                                                        const double *__restrict__ Fp, const KPoints kps,
                                                        int n_pfun, int64_t n_dof, double2 *__restrict__ f) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_pfun * n_dof) return;
    const int J = (int)(idx / n_dof);
    const int64_t i = idx - (int64_t)J * n_dof;
    double2 acc[kMaxKPerLaunch];
    for (int k = 0; k < kps.nk; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int64_t t = dof_el_off[i]; t < dof_el_off[i + 1]; ++t) {
        const int2 ea = dof_el[t];
        const ElemDev &el = elems[ea.x];
        if (el.npg == 0) continue;
        const int npad = 16 * ((el.nloc + 15) / 16);
        int corner, slot;
        local_slot(el, edof, kp.p, ea.y, &corner, &slot);
        const bool enr = ea.y >= el.nfe;
        // Bloch-periodic enrichment: periodic PU (no boundary phase on the
        // enriched rows), imaginary parts with the factor -i
        const bool imag = bpart && enr && bpart[el.edof_off + (ea.y - el.nfe)] < 0;
        const int sh_on = (bpart && enr) ? 0 : 1;
        const double *F = Fp + el.pf_base;
        for (int g = 0; g < el.npg; ++g) {
            const PGroupDev &G = pgroups[el.pg_off + g];
            const int m = J - G.J0;
            if (m < 0 || m > 2 * G.l) continue;
            const double val = F[(size_t)(G.col0 + m) * npad + ea.y];
            for (int k = 0; k < kps.nk; ++k) {
                // conj(p_a) exp(2 pi i kappa . n): phase of kappa . (n - shift_a)
                double t2 = 0.0;
                for (int d = 0; d < 3; ++d)
                    t2 += kps.kap[k][d] * (double)(G.n[d] - sh_on * ((el.shifts >> (3 * corner + d)) & 1));
                double sn, cs;
                sincos(2.0 * M_PI * t2, &sn, &cs);
                if (imag) {   // (cs + i sn)(-i val)
                    acc[k].x += sn * val;
                    acc[k].y -= cs * val;
                } else {
                    acc[k].x += cs * val;
                    acc[k].y += sn * val;
                }
            }
        }
    }
    for (int k = 0; k < kps.nk; ++k) f[((int64_t)k * n_pfun + J) * n_dof + i] = acc[k];
}

// H_ij += sum_J h_J f_J^i conj(f_J^j) over the blocks that a projector image
// couples (one work group per block), for kps.nk k-points.
__global__ __launch_bounds__(256) void nl_update_kernel(const int32_t *__restrict__ nl_blocks,
                                                        const int32_t *__restrict__ brow,
                                                        const int32_t *__restrict__ bcol,
                                                        const int64_t *__restrict__ bval_off,
                                                        const int64_t *__restrict__ dof_off,
                                                        const double2 *__restrict__ f,
                                                        const double *__restrict__ pfun_h, int n_pfun,
                                                        int64_t n_dof, int nk, int out_dtype, void *__restrict__ H,
                                                        int64_t nnz) {
    const int blk = nl_blocks[blockIdx.x];
    const int64_t v = brow[blk], w = bcol[blk];
    const int64_t r0 = dof_off[v], c0 = dof_off[w];
    const int bc = (int)(dof_off[w + 1] - c0);
    const int64_t cnt = bval_off[blk + 1] - bval_off[blk];
    for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
        const int64_t i = r0 + t / bc, j = c0 + t % bc;
        const int64_t dst = bval_off[blk] + t;
        for (int k = 0; k < nk; ++k) {
            const double2 *fk = f + (int64_t)k * n_pfun * n_dof;
            double re = 0.0, im = 0.0;
            for (int J = 0; J < n_pfun; ++J) {
                const double2 a = fk[(int64_t)J * n_dof + i], b = fk[(int64_t)J * n_dof + j];
                // h a conj(b)
                re += pfun_h[J] * (a.x * b.x + a.y * b.y);
                im += pfun_h[J] * (a.y * b.x - a.x * b.y);
            }
            if (out_dtype == 0) {
                double2 *Hk = (double2 *)H + (int64_t)k * nnz;
                double2 h = Hk[dst];
                Hk[dst] = make_double2(h.x + re, h.y + im);
            } else if (out_dtype == 1) {
                float *Hk = (float *)H + 2 * (int64_t)k * nnz;
                Hk[2 * dst] += (float)re;
                Hk[2 * dst + 1] += (float)im;
            } else {
                double *Hk = (double *)H + (int64_t)k * nnz;
                Hk[dst] += re;
            }
        }
    }
}

size_t nl_lds_bytes(int npad, int ncol, int nfun, int nimg, int nleaf, int n3) {
    return NlLds::bytes(npad, 16 * ((ncol + 15) / 16), nfun, nimg, nleaf, n3);
}

hipError_t init_nonlocal_attributes() {
    const void *ks[2] = {(const void *)nl_f_kernel<1>, (const void *)nl_f_kernel<3>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_nl_f(int lmax, const KParams &kp, int n_items, const NlItemDev *items, const ElemDev *elems,
                       const GroupDev *groups, const double *img, const int32_t *edof, const uint32_t *leaves,
                       const PGroupDev *pgroups, double *Fp, size_t lds, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (lmax <= 1)
        hipLaunchKernelGGL((nl_f_kernel<1>), dim3(n_items), dim3(kNlThreads), lds, st, kp, items, elems, groups, img,
                           edof, leaves, pgroups, Fp);
    else
        hipLaunchKernelGGL((nl_f_kernel<3>), dim3(n_items), dim3(kNlThreads), lds, st, kp, items, elems, groups, img,
                           edof, leaves, pgroups, Fp);
    return hipGetLastError();
}

hipError_t launch_nl_reduce(const ElemDev *elems, const int32_t *nl_elems, int n, double *Fp, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(nl_reduce_kernel, dim3(n), dim3(256), 0, st, elems, nl_elems, Fp);
    return hipGetLastError();
}

hipError_t launch_nl_gather(const KParams &kp, const ElemDev *elems, const PGroupDev *pgroups, const int32_t *edof,
                            const int32_t *bpart, const int64_t *dof_el_off, const int2 *dof_el, const double *Fp,
                            const KPoints &kps, int n_pfun, int64_t n_dof, double2 *f, hipStream_t st) {
    const int64_t n = (int64_t)n_pfun * n_dof;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(nl_gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kp, elems, pgroups, edof,
                       bpart, dof_el_off, dof_el, Fp, kps, n_pfun, n_dof, f);
    return hipGetLastError();
}

hipError_t launch_nl_update(int n_blocks, const int32_t *nl_blocks, const int32_t *brow, const int32_t *bcol,
                            const int64_t *bval_off, const int64_t *dof_off, const double2 *f, const double *pfun_h,
                            int n_pfun, int64_t n_dof, int nk, int out_dtype, void *H, int64_t nnz, hipStream_t st) {
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(nl_update_kernel, dim3(n_blocks), dim3(256), 0, st, nl_blocks, brow, bcol, bval_off, dof_off, f,
                       pfun_h, n_pfun, n_dof, nk, out_dtype, H, nnz);
    return hipGetLastError();
}

}  // namespace pufe
