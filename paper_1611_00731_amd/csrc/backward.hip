// Adjoint of the PUFE assembly (gfx950).
//
// For L = Re sum conj(P_ij) H_ij + Re sum conj(Q_ij) S_ij and element
// matrices H_e, S_e (eq. disceig3d), with Pt_e[a][b] = Re(p_a P[g_a][g_b] conj(p_b))
// symmetrised to Ps = (Pt + Pt^T)/2 (likewise Qs):
//   dL/dV_q  = w_q phi^T Ps phi                                    (density, eq. rhoe)
//   dL/dtau  = sum_q w_q sum_{a enriched} grad phi'_a . (Ps grad phi)_a
//              + 2 V_q phi'_a (Ps phi)_a + 2 phi'_a (Qs phi)_a
// where phi'_a = d(M_c Psi_f)/dtau = -M_c grad Psi_f.  The products
// Ps [grad phi; phi] run on FP64 MFMA; the rule, enriched sets and V are fixed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "backward.hpp"
#include "basis.hpp"
#include "device_common.hpp"
#include "tables.hpp"

namespace pufe {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Ps (or Qs) of element e into a zero-padded npad x npad row-major block.
__global__ __launch_bounds__(256) void gather_adjoint_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                             const int32_t *__restrict__ edof,
                                                             const int64_t *__restrict__ pt_off,
                                                             const double *__restrict__ Pbsr, double k0, double k1,
                                                             double k2, double *__restrict__ Pt) {
    const int e = blockIdx.x;
    const ElemDev &el = elems[e];
    const int nloc = el.nloc, npad = 16 * ((nloc + 15) / 16);
    double *dst = Pt + pt_off[e];
    for (int idx = threadIdx.x; idx < npad * npad; idx += blockDim.x) {
        const int a = idx / npad, b = idx - a * npad;
        double v = 0.0;
        if (a < nloc && b < nloc) {
            int ca, sa, cb, sb;
            local_slot(el, edof, kp.p, a, &ca, &sa);
            local_slot(el, edof, kp.p, b, &cb, &sb);
            double dn[3];
            for (int d = 0; d < 3; ++d)
                dn[d] = (double)(((el.shifts >> (3 * ca + d)) & 1) - ((el.shifts >> (3 * cb + d)) & 1));
            double sn, cs;
            sincos(2.0 * M_PI * (k0 * dn[0] + k1 * dn[1] + k2 * dn[2]), &sn, &cs);  // p_a conj(p_b)
            const int64_t oab = el.blk[ca * 8 + cb] + (int64_t)sa * el.bw[cb] + sb;
            const int64_t oba = el.blk[cb * 8 + ca] + (int64_t)sb * el.bw[ca] + sa;
            const double tab = cs * Pbsr[2 * oab] - sn * Pbsr[2 * oab + 1];
            // Re(p_b P_ba conj(p_a)): the phase is the conjugate
            const double tba = cs * Pbsr[2 * oba] + sn * Pbsr[2 * oba + 1];
            v = 0.5 * (tab + tba);
        }
        dst[idx] = v;
    }
}

// Enrichment functions of a group with gradients and Hessians:
// o[m * Q * 10 + (0 value, 1..3 gradient, 4..9 Hessian xx yy zz xy xz yz)].
// Hessian of g(s) S(r): 4 g'' r r^T S + 2 g' (S I + r grad S^T + grad S r^T) + g Hess S.
template <int L, int Q>
__device__ __forceinline__ void group_eval_hess(const GroupDev &G, const double *__restrict__ img, const double *x,
                                                double *o) {
    constexpr int NM = 2 * L + 1;
    double acc[NM][10];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int c = 0; c < 10; ++c) acc[m][c] = 0.0;
    const double rc2 = G.rc * G.rc, inv_rc2 = 1.0 / rc2;
    const double *c0 = img + 3 * G.img_off;
    for (int k = 0; k < G.nimg; ++k) {
        const double r[3] = {x[0] - c0[3 * k], x[1] - c0[3 * k + 1], x[2] - c0[3 * k + 2]};
        const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (s >= rc2) continue;
        const double ex = exp(-G.a * s), c = 1.0 - s * inv_rc2, c2 = c * c;
        const double g0 = ex * c2 * c;
        const double g1 = -ex * c2 * (G.a * c + 3.0 * inv_rc2);
        const double g2 = ex * c * (G.a * G.a * c2 + 6.0 * G.a * c * inv_rc2 + 6.0 * inv_rc2 * inv_rc2);
        double S[7], dS[21], hS[42];
        solid_harmonics(L, r[0], r[1], r[2], S, dS);
        solid_harmonics_hess(L, r[0], r[1], r[2], hS);
        const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            acc[m][0] += g0 * S[m];
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[m][1 + d] += 2.0 * g1 * r[d] * S[m] + g0 * dS[3 * m + d];
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                const int i = ii[t], j = jj[t];
                acc[m][4 + t] += 4.0 * g2 * r[i] * r[j] * S[m] +
                                 2.0 * g1 * ((i == j ? S[m] : 0.0) + r[i] * dS[3 * m + j] + dS[3 * m + i] * r[j]) +
                                 g0 * hS[6 * m + t];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int c = 0; c < 10; ++c) o[(size_t)m * Q * 10 + c] = acc[m][c];
}

template <int Q>
struct BackwardLds {
    static constexpr int RS = Q * 4 + 2;
    static __host__ __device__ size_t bytes(int npad, int nfun) {
        return sizeof(double) * ((size_t)npad * (npad + 2) + 2 * (size_t)npad * RS + (size_t)nfun * Q * 10 +
                                 (size_t)Q * 26);
    }
};

// One work group per (element, range of leaves).  QMODE = false: the P pass
// (density and the gradient/potential force terms); QMODE = true: the Q pass
// (overlap force term only).
template <int Q, bool QMODE>
__global__ __launch_bounds__(256) void backward_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, const int64_t *__restrict__ pt_off,
    const double *__restrict__ Pt, double *__restrict__ dLdV, double *__restrict__ fpart, int max_ngrp) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    constexpr int RS = BackwardLds<Q>::RS;
    const ItemDev it = items[blockIdx.x];
    const ElemDev &el = elems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun;
    const int T = (nloc + 15) / 16, npad = 16 * T, RSP = npad + 2;
    double *sP = smem;
    double *sB = sP + (size_t)npad * RSP;
    double *sU = sB + (size_t)npad * RS;
    double *sPsi = sU + (size_t)npad * RS;
    double *sQ = sPsi + (size_t)nfun * Q * 10;
    double *sXi = sQ, *sX = sQ + 3 * Q, *sW = sQ + 6 * Q, *sV = sQ + 7 * Q, *sL = sQ + 8 * Q, *sD = sQ + 17 * Q;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n3 = kp.n3;
    const int64_t q_begin = it.leaf_b * n3, q_end = it.leaf_e * n3;
    const double *src = Pt + pt_off[it.elem];
    for (int idx = tid; idx < npad * npad; idx += 256) {
        const int a = idx / npad, b = idx - a * npad;
        sP[(size_t)a * RSP + b] = src[idx];
    }
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};
    // force accumulation: thread t owns enriched row nfe + t
    const int arow = nfe + tid;
    const bool own = arow < nloc;
    int corner = 0, fidx = 0;
    if (own) {
        const int pk = edof[el.edof_off + tid];
        corner = pk & 7;
        fidx = (pk >> 3) & 255;
    }
    double facc[3] = {0.0, 0.0, 0.0};
    __syncthreads();

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
            sV[tid] = vq;
            for (int d = 0; d < 3; ++d) lagrange_1d(kp.p, xi[d], sL + 9 * tid + 3 * d, sD + 9 * tid + 3 * d);
        }
        __syncthreads();
        for (int idx = tid; idx < ngrp * Q; idx += 256) {
            const int g = idx / Q, q = idx - g * Q;
            const GroupDev G = groups[el.grp_off + g];
            double *o = sPsi + ((size_t)G.fbase * Q + q) * 10;
            switch (G.l) {
                case 0: group_eval_hess<0, Q>(G, img, sX + 3 * q, o); break;
                case 1: group_eval_hess<1, Q>(G, img, sX + 3 * q, o); break;
                case 2: group_eval_hess<2, Q>(G, img, sX + 3 * q, o); break;
                default: group_eval_hess<3, Q>(G, img, sX + 3 * q, o); break;
            }
        }
        __syncthreads();
        // basis rows (grad_x, grad_y, grad_z, value) for all local functions
        for (int idx = tid; idx < npad * Q; idx += 256) {
            const int a = idx / Q, q = idx - a * Q;
            double *o = sB + (size_t)a * RS + 4 * q;
            if (a >= nloc || sW[q] == 0.0) {
                o[0] = o[1] = o[2] = o[3] = 0.0;
                continue;
            }
            if (a < nfe) {
                const double *L = sL + 9 * q, *D = sD + 9 * q;
                const int n1 = kp.p + 1;
                const int a1 = a % n1, a2 = (a / n1) % n1, a3 = a / (n1 * n1);
                const double l1 = L[a1], l2 = L[3 + a2], l3 = L[6 + a3];
                const double dxi[3] = {D[a1] * l2 * l3, l1 * D[3 + a2] * l3, l1 * l2 * D[6 + a3]};
                for (int c = 0; c < 3; ++c)
                    o[c] = kp.Jt[3 * c] * dxi[0] + kp.Jt[3 * c + 1] * dxi[1] + kp.Jt[3 * c + 2] * dxi[2];
                o[3] = l1 * l2 * l3;
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
                const double *ps = sPsi + ((size_t)f * Q + q) * 10;
                for (int cc = 0; cc < 3; ++cc) {
                    const double gM = kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2];
                    o[cc] = gM * ps[0] + M * ps[1 + cc];
                }
                o[3] = M * ps[0];
            }
        }
        __syncthreads();
        // U[a][(q, c)] = sum_b Ps[a][b] B[b][(q, c)]: row tiles over waves,
        // K = npad in steps of 4, columns (q, c) in tiles of 16.
        {
            const int r16 = lane & 15, k4 = lane >> 4;
            for (int I = wave; I < T; I += 4) {
                for (int J = 0; J < (4 * Q) / 16; ++J) {
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
                    for (int kb = 0; kb < 4 * T; ++kb) {
                        const double a = sP[(size_t)(16 * I + r16) * RSP + 4 * kb + k4];
                        const double b = sB[(size_t)(4 * kb + k4) * RS + 16 * J + r16];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                    }
                    // FP64 16x16x4 accumulator: register r of lane l is row (l / 16) + 4 r
                    const int i0 = 16 * I + (lane >> 4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) sU[(size_t)(i0 + 4 * r) * RS + 16 * J + r16] = acc[r];
                }
            }
        }
        __syncthreads();
        if (!QMODE && dLdV != nullptr && tid < Q) {
            const int64_t qg = qb + tid;
            if (qg < q_end) {
                double s = 0.0;
                for (int a = 0; a < nloc; ++a) s += sB[(size_t)a * RS + 4 * tid + 3] * sU[(size_t)a * RS + 4 * tid + 3];
                dLdV[qg] = sW[tid] * s;
            }
        }
        if (own) {
            for (int q = 0; q < Q; ++q) {
                const double w = sW[q];
                if (w == 0.0) continue;
                double m[3], dm[3];
                for (int d = 0; d < 3; ++d) {
                    const double t = sXi[3 * q + d];
                    const int bit = (corner >> d) & 1;
                    m[d] = bit ? 0.5 * (1.0 + t) : 0.5 * (1.0 - t);
                    dm[d] = bit ? 0.5 : -0.5;
                }
                const double M = m[0] * m[1] * m[2];
                const double dM[3] = {dm[0] * m[1] * m[2], m[0] * dm[1] * m[2], m[0] * m[1] * dm[2]};
                double gM[3];
                for (int cc = 0; cc < 3; ++cc)
                    gM[cc] = kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2];
                const double *ps = sPsi + ((size_t)fidx * Q + q) * 10;
                const double gp[3] = {ps[1], ps[2], ps[3]};
                // Hessian entries H[j][k] from (xx yy zz xy xz yz)
                const double Hs[3][3] = {{ps[4], ps[7], ps[8]}, {ps[7], ps[5], ps[9]}, {ps[8], ps[9], ps[6]}};
                const double *U = sU + (size_t)arow * RS + 4 * q;
                const double u = U[3];
                for (int k = 0; k < 3; ++k) {
                    const double dphi = -M * gp[k];
                    double c;
                    if (QMODE) {
                        c = 2.0 * dphi * u;
                    } else {
                        double gg = 0.0;
                        for (int j = 0; j < 3; ++j) gg += -(gM[j] * gp[k] + M * Hs[j][k]) * U[j];
                        c = gg + 2.0 * sV[q] * dphi * u;
                    }
                    facc[k] += w * c;
                }
            }
        }
        __syncthreads();
    }
    // per-group sums of the row forces, rows in order
    double *sF = sB;
    if (own)
        for (int k = 0; k < 3; ++k) sF[3 * tid + k] = facc[k];
    __syncthreads();
    if (tid < max_ngrp) {
        double f[3] = {0.0, 0.0, 0.0};
        if (tid < ngrp) {
            const GroupDev G = groups[el.grp_off + tid];
            const int f0 = G.fbase, f1 = G.fbase + 2 * G.l + 1;
            for (int t = 0; t < nloc - nfe; ++t) {
                const int ff = (edof[el.edof_off + t] >> 3) & 255;
                if (ff >= f0 && ff < f1)
                    for (int k = 0; k < 3; ++k) f[k] += sF[3 * t + k];
            }
        }
        for (int k = 0; k < 3; ++k) fpart[((int64_t)blockIdx.x * max_ngrp + tid) * 3 + k] = f[k];
    }
}

// dL/dR of atom A: its partial slots summed in the order the host listed them
// (P pass first, then Q pass).
__global__ void force_reduce_kernel(int n_atoms, const int64_t *__restrict__ atom_ptr,
                                    const int64_t *__restrict__ atom_slots, const double *__restrict__ fpartP,
                                    const double *__restrict__ fpartQ, double *__restrict__ dLdR) {
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A >= n_atoms) return;
    double f[3] = {0.0, 0.0, 0.0};
    for (int pass = 0; pass < 2; ++pass) {
        const double *fp = pass == 0 ? fpartP : fpartQ;
        if (!fp) continue;
        for (int64_t k = atom_ptr[A]; k < atom_ptr[A + 1]; ++k) {
            const int64_t sl = atom_slots[k];
            for (int c = 0; c < 3; ++c) f[c] += fp[3 * sl + c];
        }
    }
    for (int c = 0; c < 3; ++c) dLdR[3 * A + c] = f[c];
}

hipError_t init_backward_attributes() {
    hipError_t e = hipFuncSetAttribute((const void *)backward_kernel<kBackwardQ, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)backward_kernel<kBackwardQ, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
}

size_t backward_lds_bytes(int npad, int nfun) { return BackwardLds<kBackwardQ>::bytes(npad, nfun); }

hipError_t launch_gather_adjoint(const KParams &kp, int64_t nel, const ElemDev *elems, const int32_t *edof,
                                 const int64_t *pt_off, const double *P, const double *kpt, double *Pt,
                                 hipStream_t st) {
    hipLaunchKernelGGL(gather_adjoint_kernel, dim3((unsigned)nel), dim3(256), 0, st, kp, elems, edof, pt_off, P,
                       kpt[0], kpt[1], kpt[2], Pt);
    return hipGetLastError();
}

hipError_t launch_backward(const KParams &kp, bool qmode, int n_items, const ItemDev *items, const ElemDev *elems,
                           const GroupDev *groups, const double *img, const int32_t *edof, const uint32_t *leaves,
                           const double *V, const int64_t *pt_off, const double *Pt, double *dLdV, double *fpart,
                           int max_ngrp, size_t lds, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (qmode)
        hipLaunchKernelGGL((backward_kernel<kBackwardQ, true>), dim3(n_items), dim3(256), lds, st, kp, items, elems,
                           groups, img, edof, leaves, V, pt_off, Pt, dLdV, fpart, max_ngrp);
    else
        hipLaunchKernelGGL((backward_kernel<kBackwardQ, false>), dim3(n_items), dim3(256), lds, st, kp, items, elems,
                           groups, img, edof, leaves, V, pt_off, Pt, dLdV, fpart, max_ngrp);
    return hipGetLastError();
}

hipError_t launch_force_reduce(int n_atoms, const int64_t *atom_ptr, const int64_t *atom_slots, const double *fP,
                               const double *fQ, double *dLdR, hipStream_t st) {
    if (n_atoms == 0) return hipSuccess;
    hipLaunchKernelGGL(force_reduce_kernel, dim3((n_atoms + 63) / 64), dim3(64), 0, st, n_atoms, atom_ptr,
                       atom_slots, fP, fQ, dLdR);
    return hipGetLastError();
}

}  // namespace pufe
