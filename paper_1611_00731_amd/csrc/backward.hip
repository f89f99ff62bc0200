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
#include "stage.hpp"
#include "tables.hpp"
#include "limbs.hpp"

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

// Enrichment functions of a group with gradients and Hessians at one point:
// o[(m * 10 + c) * Q], c = 0 value, 1..3 gradient, 4..9 Hessian xx yy zz xy xz yz.
// Hessian of g(s) S(r): 4 g'' r r^T S + 2 g' (S I + r grad S^T + grad S r^T) + g Hess S.
template <int L, int Q>
__device__ __forceinline__ void group_eval_hess(const GroupDev &G, const double *__restrict__ img,
                                                const double *__restrict__ spl, const double *x, double *o) {
    // the sums over images accumulate in place (the first image writes, later
    // ones add), so no per-function accumulators stay live in registers
    constexpr int NM = 2 * L + 1;
    const double rc2 = G.rc * G.rc, inv_rc2 = 1.0 / rc2;
    const double *c0 = img + 3 * G.img_off;
    bool first = true;
    for (int k = 0; k < G.nimg; ++k) {
        const double r[3] = {x[0] - c0[3 * k], x[1] - c0[3 * k + 1], x[2] - c0[3 * k + 2]};
        const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (s >= rc2) continue;
        double g0, g1, g2;
        if (G.nspl > 0) {
            spline_radial<true>(G, spl, s, g0, g1, g2);
        } else {
            const double ex = exp(-G.a * s), c = 1.0 - s * inv_rc2, c2 = c * c;
            g0 = ex * c2 * c;
            g1 = -ex * c2 * (G.a * c + 3.0 * inv_rc2);
            g2 = ex * c * (G.a * G.a * c2 + 6.0 * G.a * c * inv_rc2 + 6.0 * inv_rc2 * inv_rc2);
        }
        double S[7], dS[21], hS[42];
        solid_harmonics(L, r[0], r[1], r[2], S, dS);
        solid_harmonics_hess(L, r[0], r[1], r[2], hS);
        const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double v[10];
            v[0] = g0 * S[m];
#pragma unroll
            for (int d = 0; d < 3; ++d) v[1 + d] = 2.0 * g1 * r[d] * S[m] + g0 * dS[3 * m + d];
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                const int i = ii[t], j = jj[t];
                v[4 + t] = 4.0 * g2 * r[i] * r[j] * S[m] +
                           2.0 * g1 * ((i == j ? S[m] : 0.0) + r[i] * dS[3 * m + j] + dS[3 * m + i] * r[j]) +
                           g0 * hS[6 * m + t];
            }
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                double &oc = o[(size_t)(m * 10 + c) * Q];
                oc = first ? v[c] : oc + v[c];
            }
        }
        first = false;
    }
    if (first)
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
            for (int c = 0; c < 10; ++c) o[(size_t)(m * 10 + c) * Q] = 0.0;
}

// LDS map of the adjoint (per work item):
//   sP[npad][RSP]    Ps (or Qs) of the element, RSP = npad + 1 (FP64 form), or
//                    its bf16 limbs sPL[limb][npad][limb_row_bytes] (split form)
//   sB[npad][4][Q]   B = [d_x phi, d_y phi, d_z phi, phi] at the stage points
//   sUe[nenr][4][Q]  U = Ps B on the enriched rows (the only ones the force needs)
//   sPsi[f][10][Q]   value, gradient and Hessian of the enrichment functions
//   sGeo[GEO][Q]     per-point geometry, field-major
//   sC[r][Q][3]      force contributions of enriched row r at the stage points
//                    (in the space of sB, which is free by then)
//   sImg, sG, sEd    image centres, groups, enriched-function table
template <int Q>
struct BackwardLds {
    static constexpr int RSB = 4 * Q + 2;   // 16-byte rows
    static constexpr int GEO = 40;
    static_assert(RSB >= 3 * Q, "force contributions reuse the rows of sB");   // and stay below row nloc
    // row stride in bytes of the bf16 limbs of Ps (16-byte rows, offset banks)
    static __host__ __device__ int limb_row_bytes(int npad) { return 2 * npad + 16; }
    // doubles of the Ps region: the FP64 block, or up to three limb blocks
    static __host__ __device__ size_t p_doubles(int npad) {
        const size_t f = (size_t)npad * (npad + 1), l = (3 * (size_t)npad * limb_row_bytes(npad) + 7) / 8;
        return f > l ? f : l;
    }
    static __host__ __device__ size_t bytes(int npad, int nenr, int nfun, int nimg) {
        return sizeof(double) * (p_doubles(npad) + (size_t)npad * RSB + (size_t)nenr * RSB +
                                 (size_t)nfun * Q * 10 + (size_t)Q * GEO + (size_t)nimg * 3) +
               sizeof(GroupDev) * kMaxGroups + sizeof(int32_t) * (kMaxNloc + 16) + 64;
    }
};

// geometry fields (index f at sGeo[f * Q + q])
enum { B_XI = 0, B_X = 3, B_W = 6, B_V = 7, B_L = 8, B_D = 17, B_M = 26, B_M1 = 34 };
// the shape-function fields sit where the grouped row helpers read them, and
// the weight at the field those helpers test in their unweighted form
static_assert(B_L == G_L && B_D == G_D && B_M == G_M && B_M1 == G_M1 && B_W == 6, "geometry layout");

// U = Ps B for operand component c (one per wave), all T row tiles at once:
// output tile I covers rows 16 I .. 16 I + 15 and the Q = 16 stage points of
// component c, K = npad.  The U rows of the enriched functions go to sUe; the
// wave holding the value component (c = 3) also forms the density
// dL/dV_q = w_q sum_a phi_a (Ps phi)_a from its accumulators.
template <int T, int Q, bool DENS>
__device__ __forceinline__ void backward_mfma(const double *__restrict__ sP, const double *__restrict__ sB,
                                              double *__restrict__ sUe, const double *__restrict__ sGeo, int RSP,
                                              int nloc, int nfe, int c, int lane, int64_t qb, int64_t q_end,
                                              double *__restrict__ dLdV) {
    static_assert(Q == 16, "one output tile spans the stage");
    constexpr int RSB = BackwardLds<Q>::RSB;
    const int r16 = lane & 15, k4 = lane >> 4;
    double4_t acc[T];
#pragma unroll
    for (int I = 0; I < T; ++I) acc[I] = (double4_t){0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < 4 * T; ++kb) {
        const double b = sB[(size_t)(4 * kb + k4) * RSB + c * Q + r16];
        double a[T];
#pragma unroll
        for (int I = 0; I < T; ++I) a[I] = sP[(size_t)(16 * I + r16) * RSP + 4 * kb + k4];
#pragma unroll
        for (int I = 0; I < T; ++I) acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], b, acc[I], 0, 0, 0);
    }
    // FP64 16x16x4 accumulator: register r of lane l is row (l / 16) + 4 r, column (point) l % 16
    double dens = 0.0;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * I + k4 + 4 * r;
            if (row >= nfe && row < nloc) sUe[(size_t)(row - nfe) * RSB + c * Q + r16] = acc[I][r];
            if (DENS && row < nloc) dens += sB[(size_t)row * RSB + 3 * Q + r16] * acc[I][r];
        }
    if (DENS) {
        dens += __shfl_xor(dens, 16, 64);
        dens += __shfl_xor(dens, 32, 64);
        const int64_t qg = qb + r16;
        if (k4 == 0 && qg < q_end) dLdV[qg] = sGeo[B_W * Q + r16] * dens;
    }
}

// Split-precision form of backward_mfma: Ps comes as NL bf16 limbs (split
// once per item), B is split into limbs in registers as its FP64 rows are
// read, and U = Ps B is summed from the kept limb products on
// v_mfma_f32_16x16x32_bf16 in FP32, K-blocks of 32 functions (the block past
// npad reads zeros).  Lane l = i + 16 g supplies row i of the A tile at
// functions 8 g .. 8 g + 7 of the block and those functions at point i of B;
// result register r of lane l is row 4 (l / 16) + r, point l % 16.
template <int T, int Q, bool DENS, int NL>
__device__ __forceinline__ void backward_mfma_split(const unsigned char *__restrict__ sPL, const double *__restrict__ sB,
                                                    double *__restrict__ sUe, const double *__restrict__ sGeo,
                                                    int RSP, int nloc, int nfe, int c, int lane, int64_t qb,
                                                    int64_t q_end, double *__restrict__ dLdV) {
    static_assert(Q == 16, "one output tile spans the stage");
    constexpr int RSB = BackwardLds<Q>::RSB;
    constexpr int npad = 16 * T;
    const int r16 = lane & 15, g4 = lane >> 4;
    f32x4 acc[T];
#pragma unroll
    for (int I = 0; I < T; ++I) acc[I] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < npad; kb += 32) {
        const int b0 = kb + 8 * g4;
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = b0 + i < npad ? sB[(size_t)(b0 + i) * RSB + c * Q + r16] : 0.0;
        bf16x8 Bl[NL];
        split_limbs8<NL>(v, Bl);
        const int RPL = BackwardLds<Q>::limb_row_bytes(npad);
#pragma unroll
        for (int I = 0; I < T; ++I) {
            bf16x8 Al[NL];
#pragma unroll
            for (int j = 0; j < NL; ++j)
                Al[j] = b0 < npad ? *(const bf16x8 *)(sPL + ((size_t)j * npad + 16 * I + r16) * RPL + 2 * b0)
                                  : (bf16x8){};
            acc[I] = mfma_limbs<NL>(Al, Bl, acc[I]);
        }
    }
    double dens = 0.0;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * I + 4 * g4 + r;
            const double u = (double)acc[I][r];
            if (row >= nfe && row < nloc) sUe[(size_t)(row - nfe) * RSB + c * Q + r16] = u;
            if (DENS && row < nloc) dens += sB[(size_t)row * RSB + 3 * Q + r16] * u;
        }
    if (DENS) {
        dens += __shfl_xor(dens, 16, 64);
        dens += __shfl_xor(dens, 32, 64);
        const int64_t qg = qb + r16;
        if (g4 == 0 && qg < q_end) dLdV[qg] = sGeo[B_W * Q + r16] * dens;
    }
}

template <int Q, bool DENS, int NL>
__device__ __forceinline__ void backward_mfma_dispatch(int T, const double *sP, const double *sB, double *sUe,
                                                       const double *sGeo, int RSP, int nloc, int nfe, int c,
                                                       int lane, int64_t qb, int64_t q_end, double *dLdV) {
#define PUFE_BWM(TT)                                                                                     \
    if constexpr (NL == 0)                                                                               \
        backward_mfma<TT, Q, DENS>(sP, sB, sUe, sGeo, RSP, nloc, nfe, c, lane, qb, q_end, dLdV);         \
    else                                                                                                 \
        backward_mfma_split<TT, Q, DENS, NL>((const unsigned char *)sP, sB, sUe, sGeo, RSP, nloc, nfe, c, lane, qb, \
                                             q_end, dLdV)
    switch (T) {
        case 1: PUFE_BWM(1); break;
        case 2: PUFE_BWM(2); break;
        case 3: PUFE_BWM(3); break;
        case 4: PUFE_BWM(4); break;
        default: PUFE_BWM(5); break;
    }
#undef PUFE_BWM
}

// One work group per (element, range of leaves).  QMODE = false: the P pass
// (density and the gradient/potential force terms); QMODE = true: the Q pass
// (overlap force term only).  NL = 0: U = Ps B on FP64 MFMAs; NL = 2 or 3:
// split-precision U from 2 or 3 bf16 limbs per operand (bf16x3, bf16x6).
template <int Q, bool QMODE, int NL>
__global__ __launch_bounds__(256) void backward_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, const int64_t *__restrict__ pt_off,
    const double *__restrict__ Pt, double *__restrict__ dLdV, double *__restrict__ fpart, int max_ngrp) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    constexpr int RSB = BackwardLds<Q>::RSB;
    constexpr int NT = 256;
    const ItemDev it = items[blockIdx.x];
    const ElemDev &el = elems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun, nenr = nloc - nfe;
    const int T = (nloc + 15) / 16, npad = 16 * T, RSP = npad + 1;
    const int img0 = ngrp > 0 ? groups[el.grp_off].img_off : 0;
    const int nimg = ngrp > 0 ? groups[el.grp_off + ngrp - 1].img_off + groups[el.grp_off + ngrp - 1].nimg - img0 : 0;
    double *sP = smem;
    double *sB = sP + BackwardLds<Q>::p_doubles(npad);
    double *sUe = sB + (size_t)npad * RSB;
    double *sPsi = sUe + (size_t)nenr * RSB;
    double *sGeo = sPsi + (size_t)nfun * Q * 10;
    double *sC = sB;   // [nenr][Q][3], written after the MFMA phase has read sB
    double *sImg = sGeo + (size_t)Q * BackwardLds<Q>::GEO;
    GroupDev *sG = (GroupDev *)(sImg + 3 * (size_t)nimg);
    int32_t *sEd = (int32_t *)(sG + kMaxGroups);
    int *sCS = sEd + kMaxNloc;   // [9] PU corner starts in sEd
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n3 = kp.n3;
    const int64_t q_begin = it.leaf_b * n3, q_end = it.leaf_e * n3;
    const double *src = Pt + pt_off[it.elem];
    if constexpr (NL == 0) {
        for (int idx = tid; idx < npad * npad; idx += NT) {
            const int a = idx / npad, b = idx - a * npad;
            sP[(size_t)a * RSP + b] = src[idx];
        }
    } else {
        // bf16 limbs of Ps, split once per item (two adjacent entries per thread)
        unsigned char *sPL = (unsigned char *)sP;
        const int RPL = BackwardLds<Q>::limb_row_bytes(npad), hp = npad / 2;
        for (int idx = tid; idx < npad * hp; idx += NT) {
            const int a = idx / hp, b = 2 * (idx - a * hp);
            uint32_t h[NL];
            split_limbs2<NL>(src[(size_t)a * npad + b], src[(size_t)a * npad + b + 1], h);
#pragma unroll
            for (int j = 0; j < NL; ++j) *(uint32_t *)(sPL + ((size_t)j * npad + a) * RPL + 2 * b) = h[j];
        }
    }
    for (int k = tid; k < nenr; k += NT) sEd[k] = edof[el.edof_off + k];
    corner_starts((const PUFE_GLOBAL int32_t *)(edof + el.edof_off), nenr, sCS, tid, NT);
    // the padding rows of B stay zero (the force buffer sC lies within the
    // first nloc rows)
    for (int k = tid; k < (npad - nloc) * RSB; k += NT) sB[(size_t)nloc * RSB + k] = 0.0;
    for (int g = tid; g < ngrp; g += NT) {
        GroupDev G = groups[el.grp_off + g];
        G.img_off -= img0;   // rebased onto sImg
        sG[g] = G;
    }
    for (int k = tid; k < 3 * nimg; k += NT) sImg[k] = img[3 * (size_t)img0 + k];
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};
    const KLocal kl = load_klocal(kp);
    // force accumulation: thread t owns enriched row nfe + t (rows of one
    // stage are summed over its points in order, then over the stages)
    double facc[3] = {0.0, 0.0, 0.0};
    const int gq = tid - (NT - Q);   // the last Q threads build the geometry
    __syncthreads();

    for (int64_t qb = q_begin; qb < q_end; qb += Q) {
        // ---- phase 1: geometry, enrichment functions with Hessians, and the
        // previous stage's force contributions folded into the row sums
        if (tid < nenr && qb > q_begin)
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int k = 0; k < 3; ++k) facc[k] += sC[((size_t)tid * Q + q) * 3 + k];
        if (gq >= 0) {
            const int64_t qg = qb + gq;
            double xi[3] = {0.0, 0.0, 0.0}, w = 0.0, vq = 0.0;
            if (qg < q_end) {
                const int64_t lf = qg / n3;
                leaf_point(kp, leaves[lf], (int)(qg - lf * n3), xi, &w);
                vq = V[qg];
            }
            double *g = sGeo + gq;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                g[(B_XI + d) * Q] = xi[d];
                g[(B_X + d) * Q] = org[d] + 0.5 * (xi[0] + 1.0) * kp.E[d] + 0.5 * (xi[1] + 1.0) * kp.E[3 + d] +
                                   0.5 * (xi[2] + 1.0) * kp.E[6 + d];
            }
            g[B_W * Q] = w;
            g[B_V * Q] = vq;
            double Lv[9], Dv[9];
            for (int d = 0; d < 3; ++d) lagrange_1d(kp.p, xi[d], Lv + 3 * d, Dv + 3 * d);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                g[(B_L + k) * Q] = Lv[k];
                g[(B_D + k) * Q] = Dv[k];
            }
            double m[3][2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                m[d][0] = 0.5 * (1.0 - xi[d]);
                m[d][1] = 0.5 * (1.0 + xi[d]);
                g[(B_M1 + 2 * d) * Q] = m[d][0];
                g[(B_M1 + 2 * d + 1) * Q] = m[d][1];
            }
#pragma unroll
            for (int c8 = 0; c8 < 8; ++c8) g[(B_M + c8) * Q] = m[0][c8 & 1] * m[1][(c8 >> 1) & 1] * m[2][c8 >> 2];
        }
        for (int idx = tid; idx < ngrp * Q; idx += NT) {
            const int gi = idx / Q, q = idx - gi * Q;
            const GroupDev &G = sG[gi];
            const int64_t qg = qb + q;
            double xi[3] = {0.0, 0.0, 0.0}, w = 0.0, x[3];
            if (qg < q_end) {
                const int64_t lf = qg / n3;
                leaf_point(kp, leaves[lf], (int)(qg - lf * n3), xi, &w);
            }
            for (int d = 0; d < 3; ++d)
                x[d] = org[d] + 0.5 * (xi[0] + 1.0) * kp.E[d] + 0.5 * (xi[1] + 1.0) * kp.E[3 + d] +
                       0.5 * (xi[2] + 1.0) * kp.E[6 + d];
            double *o = sPsi + (size_t)G.fbase * 10 * Q + q;
            switch (G.l) {
                case 0: group_eval_hess<0, Q>(G, sImg, kp.spl, x, o); break;
                case 1: group_eval_hess<1, Q>(G, sImg, kp.spl, x, o); break;
                case 2: group_eval_hess<2, Q>(G, sImg, kp.spl, x, o); break;
                default: group_eval_hess<3, Q>(G, sImg, kp.spl, x, o); break;
            }
        }
        __syncthreads();
        // ---- phase 2: basis rows (grad_x, grad_y, grad_z, value), unweighted
        // (zero past the item's last point), in groups sharing the point's
        // geometry: FE functions by (a2, a3), enriched ones by PU corner
        {
            const int nfu = fe_units(kl.p);
            for (int idx = tid; idx < (nfu + 8) * Q; idx += NT) {
                const int u = idx / Q, q = idx - u * Q;
                double *o = sB + q;
                auto put = [&](int a, double x, double y, double z, double w) {
                    double *r = o + (size_t)a * RSB;
                    r[0] = x;
                    r[Q] = y;
                    r[2 * Q] = z;
                    r[3 * Q] = w;
                };
                if (u >= nfu) {
                    const int c = u - nfu;
                    pu_unit<Q, 10 * Q, true>(kl, sGeo + q, sPsi + q, sEd, c, sCS[c], sCS[c + 1], nfe, put);
                } else {
                    fe_unit_any<Q, true>(kl, sGeo + q, u, put);
                }
            }
        }
        __syncthreads();
        // ---- phase 3: U = Ps B on the MFMAs, one operand component per wave;
        // the value component also gives the density
        if (!QMODE && dLdV != nullptr && wave == 3)
            backward_mfma_dispatch<Q, true, NL>(T, sP, sB, sUe, sGeo, RSP, nloc, nfe, wave, lane, qb, q_end, dLdV);
        else
            backward_mfma_dispatch<Q, false, NL>(T, sP, sB, sUe, sGeo, RSP, nloc, nfe, wave, lane, qb, q_end, dLdV);
        __syncthreads();
        // ---- phase 4: force contributions of every (enriched row, point)
        for (int idx = tid; idx < nenr * Q; idx += NT) {
            const int r = idx / Q, q = idx - r * Q;
            const double *g = sGeo + q;
            const double w = g[B_W * Q];
            double cf[3] = {0.0, 0.0, 0.0};
            if (w != 0.0) {
                const int pk = sEd[r];
                const int corner = pk & 7, f = (pk >> 3) & 255;
                const int b0 = corner & 1, b1 = (corner >> 1) & 1, b2 = corner >> 2;
                const double m0 = g[(B_M1 + b0) * Q], m1 = g[(B_M1 + 2 + b1) * Q], m2 = g[(B_M1 + 4 + b2) * Q];
                const double M = g[(B_M + corner) * Q];
                const double dM[3] = {(b0 ? 0.5 : -0.5) * m1 * m2, m0 * (b1 ? 0.5 : -0.5) * m2,
                                      m0 * m1 * (b2 ? 0.5 : -0.5)};
                double gM[3];
                for (int cc = 0; cc < 3; ++cc)
                    gM[cc] = kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2];
                const double *ps = sPsi + (size_t)f * 10 * Q + q;
                const double gp[3] = {ps[Q], ps[2 * Q], ps[3 * Q]};
                // Hessian entries H[j][k] from (xx yy zz xy xz yz)
                const double Hs[3][3] = {{ps[4 * Q], ps[7 * Q], ps[8 * Q]},
                                         {ps[7 * Q], ps[5 * Q], ps[9 * Q]},
                                         {ps[8 * Q], ps[9 * Q], ps[6 * Q]}};
                const double *U = sUe + (size_t)r * RSB + q;
                const double u = U[3 * Q];
                for (int k = 0; k < 3; ++k) {
                    const double dphi = -M * gp[k];   // d phi'/d tau_k
                    double c;
                    if (QMODE) {
                        c = 2.0 * dphi * u;
                    } else {
                        double gg = 0.0;
                        for (int jj = 0; jj < 3; ++jj) gg += -(gM[jj] * gp[k] + M * Hs[jj][k]) * U[jj * Q];
                        c = gg + 2.0 * g[B_V * Q] * dphi * u;
                    }
                    cf[k] = w * c;
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) sC[((size_t)r * Q + q) * 3 + k] = cf[k];
        }
        __syncthreads();
    }
    if (tid < nenr && q_end > q_begin)
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) facc[k] += sC[((size_t)tid * Q + q) * 3 + k];
    // per-group sums of the row forces, rows in order
    double *sF = sB;
    __syncthreads();
    if (tid < nenr)
        for (int k = 0; k < 3; ++k) sF[3 * tid + k] = facc[k];
    __syncthreads();
    if (tid < max_ngrp) {
        double f[3] = {0.0, 0.0, 0.0};
        if (tid < ngrp) {
            const GroupDev G = sG[tid];
            const int f0 = G.fbase, f1 = G.fbase + 2 * G.l + 1;
            for (int t = 0; t < nenr; ++t) {
                const int ff = (sEd[t] >> 3) & 255;
                if (ff >= f0 && ff < f1)
                    for (int k = 0; k < 3; ++k) f[k] += sF[3 * t + k];
            }
        }
        for (int k = 0; k < 3; ++k) fpart[((int64_t)blockIdx.x * max_ngrp + tid) * 3 + k] = f[k];
    }
}

// Elements of more than 80 functions (FP64).  Their block of Ps does not fit
// in LDS, so each stage walks the row blocks R of kBwBlock functions and, for
// each, the column blocks K (R last): Ps[R][K] is copied into LDS, the rows of
// K are evaluated, and U[R] += Ps[R][K] B[K] accumulates on the MFMAs (one
// operand component per wave, as in backward_kernel).  With K = R last, sB
// holds R's own rows when U[R] is complete: the value-component wave adds
// sum_{a in R} phi_a U_a to the point's density, U of R's enriched rows goes
// to LDS, and the force contributions of those rows follow.  Thread t owns
// enriched row nfe + t (the host admits at most 256 enriched functions).
//   sP  [kBwBlock][RSB]   Ps[R][K], then U of R's enriched rows
//   sB  [kBwBlock][RSB]   B rows of K, then the force contributions sC
//   sPsi, sGeo, sImg, sG, sEd, sCS as in backward_kernel
template <bool QMODE>
__global__ __launch_bounds__(256) void backward_wide_kernel(
    const KParams kp, const ItemDev *__restrict__ items, const ElemDev *__restrict__ elems,
    const GroupDev *__restrict__ groups, const double *__restrict__ img, const int32_t *__restrict__ edof,
    const uint32_t *__restrict__ leaves, const double *__restrict__ V, const int64_t *__restrict__ pt_off,
    const double *__restrict__ Pt, double *__restrict__ dLdV, double *__restrict__ fpart, int max_ngrp) {
    extern __shared__ __attribute__((aligned(16))) double smem[];
    constexpr int Q = kBackwardQ;
    constexpr int RSB = BackwardLds<Q>::RSB;
    constexpr int NT = 256, BK = kBwBlock, TB = BK / 16;
    const ItemDev it = items[blockIdx.x];
    const ElemDev &el = elems[it.elem];
    const int nloc = el.nloc, nfe = el.nfe, ngrp = el.ngrp, nfun = el.nfun, nenr = nloc - nfe;
    const int npad = 16 * ((nloc + 15) / 16), nb = (nloc + BK - 1) / BK;
    const int img0 = ngrp > 0 ? groups[el.grp_off].img_off : 0;
    const int nimg = ngrp > 0 ? groups[el.grp_off + ngrp - 1].img_off + groups[el.grp_off + ngrp - 1].nimg - img0 : 0;
    double *sP = smem;
    double *sB = sP + (size_t)BK * RSB;
    double *sPsi = sB + (size_t)BK * RSB;
    double *sGeo = sPsi + (size_t)nfun * Q * 10;
    double *sImg = sGeo + (size_t)Q * BackwardLds<Q>::GEO;
    GroupDev *sG = (GroupDev *)(sImg + 3 * (size_t)nimg);
    int32_t *sEd = (int32_t *)(sG + kMaxGroups);
    int *sCS = sEd + kMaxNloc;
    double *sUe = sP;   // after a row block's column loop
    double *sC = sB;    // [BK][Q][3], after the density has read sB
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int n3 = kp.n3;
    const int64_t q_begin = it.leaf_b * n3, q_end = it.leaf_e * n3;
    const double *src = Pt + pt_off[it.elem];
    for (int k = tid; k < nenr; k += NT) sEd[k] = edof[el.edof_off + k];
    corner_starts((const PUFE_GLOBAL int32_t *)(edof + el.edof_off), nenr, sCS, tid, NT);
    for (int g = tid; g < ngrp; g += NT) {
        GroupDev G = groups[el.grp_off + g];
        G.img_off -= img0;   // rebased onto sImg
        sG[g] = G;
    }
    for (int k = tid; k < 3 * nimg; k += NT) sImg[k] = img[3 * (size_t)img0 + k];
    const double org[3] = {el.ijk[0] * kp.E[0] + el.ijk[1] * kp.E[3] + el.ijk[2] * kp.E[6],
                           el.ijk[0] * kp.E[1] + el.ijk[1] * kp.E[4] + el.ijk[2] * kp.E[7],
                           el.ijk[0] * kp.E[2] + el.ijk[1] * kp.E[5] + el.ijk[2] * kp.E[8]};
    const KLocal kl = load_klocal(kp);
    const int nfu = fe_units(kl.p);
    double facc[3] = {0.0, 0.0, 0.0};   // forces of enriched row nfe + tid
    const int gq = tid - (NT - Q);
    __syncthreads();

    for (int64_t qb = q_begin; qb < q_end; qb += Q) {
        // ---- phase 1: geometry, enrichment functions with Hessians
        if (gq >= 0) {
            const int64_t qg = qb + gq;
            double xi[3] = {0.0, 0.0, 0.0}, w = 0.0, vq = 0.0;
            if (qg < q_end) {
                const int64_t lf = qg / n3;
                leaf_point(kp, leaves[lf], (int)(qg - lf * n3), xi, &w);
                vq = V[qg];
            }
            double *g = sGeo + gq;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                g[(B_XI + d) * Q] = xi[d];
                g[(B_X + d) * Q] = org[d] + 0.5 * (xi[0] + 1.0) * kp.E[d] + 0.5 * (xi[1] + 1.0) * kp.E[3 + d] +
                                   0.5 * (xi[2] + 1.0) * kp.E[6 + d];
            }
            g[B_W * Q] = w;
            g[B_V * Q] = vq;
            double Lv[9], Dv[9];
            for (int d = 0; d < 3; ++d) lagrange_1d(kp.p, xi[d], Lv + 3 * d, Dv + 3 * d);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                g[(B_L + k) * Q] = Lv[k];
                g[(B_D + k) * Q] = Dv[k];
            }
            double m[3][2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                m[d][0] = 0.5 * (1.0 - xi[d]);
                m[d][1] = 0.5 * (1.0 + xi[d]);
                g[(B_M1 + 2 * d) * Q] = m[d][0];
                g[(B_M1 + 2 * d + 1) * Q] = m[d][1];
            }
#pragma unroll
            for (int c8 = 0; c8 < 8; ++c8) g[(B_M + c8) * Q] = m[0][c8 & 1] * m[1][(c8 >> 1) & 1] * m[2][c8 >> 2];
        }
        for (int idx = tid; idx < ngrp * Q; idx += NT) {
            const int gi = idx / Q, q = idx - gi * Q;
            const GroupDev &G = sG[gi];
            const int64_t qg = qb + q;
            double xi[3] = {0.0, 0.0, 0.0}, w = 0.0, x[3];
            if (qg < q_end) {
                const int64_t lf = qg / n3;
                leaf_point(kp, leaves[lf], (int)(qg - lf * n3), xi, &w);
            }
            for (int d = 0; d < 3; ++d)
                x[d] = org[d] + 0.5 * (xi[0] + 1.0) * kp.E[d] + 0.5 * (xi[1] + 1.0) * kp.E[3 + d] +
                       0.5 * (xi[2] + 1.0) * kp.E[6 + d];
            double *o = sPsi + (size_t)G.fbase * 10 * Q + q;
            switch (G.l) {
                case 0: group_eval_hess<0, Q>(G, sImg, kp.spl, x, o); break;
                case 1: group_eval_hess<1, Q>(G, sImg, kp.spl, x, o); break;
                case 2: group_eval_hess<2, Q>(G, sImg, kp.spl, x, o); break;
                default: group_eval_hess<3, Q>(G, sImg, kp.spl, x, o); break;
            }
        }
        __syncthreads();
        double dens = 0.0;   // wave 3: its lanes' share of phi^T Ps phi at point r16
        for (int rb = 0; rb < nb; ++rb) {
            const int r0 = rb * BK, r1 = min(r0 + BK, nloc);
            double4_t acc[TB];
#pragma unroll
            for (int I = 0; I < TB; ++I) acc[I] = (double4_t){0.0, 0.0, 0.0, 0.0};
            for (int j = 1; j <= nb; ++j) {
                const int kb = (rb + j) % nb;   // the row block itself comes last
                const int k0 = kb * BK, k1 = min(k0 + BK, nloc), nkp = 16 * ((k1 - k0 + 15) / 16);
                // Ps[R][K] (zero past the padded block), and the rows of K (zero past k1)
                for (int idx = tid; idx < BK * BK; idx += NT) {
                    const int a = idx / BK, b = idx - a * BK;
                    const int ga = r0 + a, gb = k0 + b;
                    sP[(size_t)a * RSB + b] = (ga < npad && gb < npad) ? src[(size_t)ga * npad + gb] : 0.0;
                }
                for (int k = tid; k < (BK - (k1 - k0)) * RSB; k += NT) sB[(size_t)(k1 - k0) * RSB + k] = 0.0;
                {
                    // FE units when K holds FE rows, then the corner runs of K's enriched rows
                    const int nu_fe = k0 < nfe ? nfu : 0;
                    for (int idx = tid; idx < (nu_fe + 8) * Q; idx += NT) {
                        const int u = idx / Q, q = idx - u * Q;
                        double *o = sB + q;
                        auto put = [&](int a, double x, double y, double z, double w) {
                            if (a < k0 || a >= k1) return;
                            double *r = o + (size_t)(a - k0) * RSB;
                            r[0] = x;
                            r[Q] = y;
                            r[2 * Q] = z;
                            r[3 * Q] = w;
                        };
                        if (u < nu_fe) {
                            fe_unit_any<Q, true>(kl, sGeo + q, u, put);
                        } else {
                            const int c = u - nu_fe;
                            const int kb0 = max(sCS[c], k0 - nfe), kb1 = min(sCS[c + 1], k1 - nfe);
                            if (kb0 < kb1)
                                pu_unit<Q, 10 * Q, true>(kl, sGeo + q, sPsi + q, sEd, c, kb0, kb1, nfe, put);
                        }
                    }
                }
                __syncthreads();
                // U[R] += Ps[R][K] B[K], component `wave`
                for (int kk = 0; kk < nkp; kk += 4) {
                    const double b = sB[(size_t)(kk + k4) * RSB + wave * Q + r16];
#pragma unroll
                    for (int I = 0; I < TB; ++I) {
                        const double a = sP[(size_t)(16 * I + r16) * RSB + kk + k4];
                        acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[I], 0, 0, 0);
                    }
                }
                __syncthreads();
            }
            // sB now holds R's own rows: density, then U of R's enriched rows
            // (register r of lane l is row (l / 16) + 4 r of the tile, point l % 16)
            if (!QMODE && wave == 3)
#pragma unroll
                for (int I = 0; I < TB; ++I)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * I + k4 + 4 * r;
                        if (r0 + row < r1) dens += sB[(size_t)row * RSB + 3 * Q + r16] * acc[I][r];
                    }
#pragma unroll
            for (int I = 0; I < TB; ++I)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + k4 + 4 * r;
                    if (r0 + row >= nfe && r0 + row < r1) sUe[(size_t)row * RSB + wave * Q + r16] = acc[I][r];
                }
            __syncthreads();
            // force contributions of every (enriched row of R, point)
            const int e0 = max(r0, nfe);
            for (int idx = tid; idx < (r1 - e0) * Q; idx += NT) {
                const int ra = e0 + idx / Q, q = idx % Q, rl = ra - r0;
                const double *g = sGeo + q;
                const double w = g[B_W * Q];
                double cf[3] = {0.0, 0.0, 0.0};
                if (w != 0.0) {
                    const int pk = sEd[ra - nfe];
                    const int corner = pk & 7, f = (pk >> 3) & 255;
                    const int b0 = corner & 1, b1 = (corner >> 1) & 1, b2 = corner >> 2;
                    const double m0 = g[(B_M1 + b0) * Q], m1 = g[(B_M1 + 2 + b1) * Q], m2 = g[(B_M1 + 4 + b2) * Q];
                    const double M = g[(B_M + corner) * Q];
                    const double dM[3] = {(b0 ? 0.5 : -0.5) * m1 * m2, m0 * (b1 ? 0.5 : -0.5) * m2,
                                          m0 * m1 * (b2 ? 0.5 : -0.5)};
                    double gM[3];
                    for (int cc = 0; cc < 3; ++cc)
                        gM[cc] = kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2];
                    const double *ps = sPsi + (size_t)f * 10 * Q + q;
                    const double gp[3] = {ps[Q], ps[2 * Q], ps[3 * Q]};
                    const double Hs[3][3] = {{ps[4 * Q], ps[7 * Q], ps[8 * Q]},
                                             {ps[7 * Q], ps[5 * Q], ps[9 * Q]},
                                             {ps[8 * Q], ps[9 * Q], ps[6 * Q]}};
                    const double *U = sUe + (size_t)rl * RSB + q;
                    const double u = U[3 * Q];
                    for (int k = 0; k < 3; ++k) {
                        const double dphi = -M * gp[k];
                        double c;
                        if (QMODE) {
                            c = 2.0 * dphi * u;
                        } else {
                            double gg = 0.0;
                            for (int jj = 0; jj < 3; ++jj) gg += -(gM[jj] * gp[k] + M * Hs[jj][k]) * U[jj * Q];
                            c = gg + 2.0 * g[B_V * Q] * dphi * u;
                        }
                        cf[k] = w * c;
                    }
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) sC[((size_t)rl * Q + q) * 3 + k] = cf[k];
            }
            __syncthreads();
            {
                const int ra = nfe + tid;
                if (tid < nenr && ra >= r0 && ra < r1)
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int k = 0; k < 3; ++k) facc[k] += sC[((size_t)(ra - r0) * Q + q) * 3 + k];
            }
            __syncthreads();
        }
        if (!QMODE && dLdV != nullptr && wave == 3) {
            dens += __shfl_xor(dens, 16, 64);
            dens += __shfl_xor(dens, 32, 64);
            const int64_t qg = qb + r16;
            if (k4 == 0 && qg < q_end) dLdV[qg] = sGeo[B_W * Q + r16] * dens;
        }
        __syncthreads();
    }
    // per-group sums of the row forces, rows in order
    double *sF = sB;
    if (tid < nenr)
        for (int k = 0; k < 3; ++k) sF[3 * tid + k] = facc[k];
    __syncthreads();
    if (tid < max_ngrp) {
        double f[3] = {0.0, 0.0, 0.0};
        if (tid < ngrp) {
            const GroupDev G = sG[tid];
            const int f0 = G.fbase, f1 = G.fbase + 2 * G.l + 1;
            for (int t = 0; t < nenr; ++t) {
                const int ff = (sEd[t] >> 3) & 255;
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
    const void *ks[8] = {(const void *)backward_kernel<kBackwardQ, false, 0>,
                         (const void *)backward_kernel<kBackwardQ, true, 0>,
                         (const void *)backward_kernel<kBackwardQ, false, 2>,
                         (const void *)backward_kernel<kBackwardQ, true, 2>,
                         (const void *)backward_kernel<kBackwardQ, false, 3>,
                         (const void *)backward_kernel<kBackwardQ, true, 3>,
                         (const void *)backward_wide_kernel<false>,
                         (const void *)backward_wide_kernel<true>};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t backward_lds_bytes(int npad, int nenr, int nfun, int nimg) {
    return BackwardLds<kBackwardQ>::bytes(npad, nenr, nfun, nimg);
}

size_t backward_wide_lds_bytes(int nfun, int nimg) {
    constexpr int Q = kBackwardQ;
    return sizeof(double) * (2 * (size_t)kBwBlock * BackwardLds<Q>::RSB + (size_t)nfun * Q * 10 +
                             (size_t)Q * BackwardLds<Q>::GEO + (size_t)nimg * 3) +
           sizeof(GroupDev) * kMaxGroups + sizeof(int32_t) * (kMaxNloc + 16) + 64;
}

hipError_t launch_backward_wide(const KParams &kp, bool qmode, int n_items, const ItemDev *items,
                                const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                                const uint32_t *leaves, const double *V, const int64_t *pt_off, const double *Pt,
                                double *dLdV, double *fpart, int max_ngrp, size_t lds, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (qmode)
        hipLaunchKernelGGL((backward_wide_kernel<true>), dim3(n_items), dim3(256), lds, st, kp, items, elems, groups,
                           img, edof, leaves, V, pt_off, Pt, dLdV, fpart, max_ngrp);
    else
        hipLaunchKernelGGL((backward_wide_kernel<false>), dim3(n_items), dim3(256), lds, st, kp, items, elems, groups,
                           img, edof, leaves, V, pt_off, Pt, dLdV, fpart, max_ngrp);
    return hipGetLastError();
}

hipError_t launch_gather_adjoint(const KParams &kp, int64_t nel, const ElemDev *elems, const int32_t *edof,
                                 const int64_t *pt_off, const double *P, const double *kpt, double *Pt,
                                 hipStream_t st) {
    hipLaunchKernelGGL(gather_adjoint_kernel, dim3((unsigned)nel), dim3(256), 0, st, kp, elems, edof, pt_off, P,
                       kpt[0], kpt[1], kpt[2], Pt);
    return hipGetLastError();
}

hipError_t launch_backward(const KParams &kp, bool qmode, int nl, int n_items, const ItemDev *items,
                           const ElemDev *elems, const GroupDev *groups, const double *img, const int32_t *edof,
                           const uint32_t *leaves, const double *V, const int64_t *pt_off, const double *Pt,
                           double *dLdV, double *fpart, int max_ngrp, size_t lds, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (nl != 0 && nl != 2 && nl != 3) return hipErrorInvalidValue;
#define PUFE_BWK(QM, NLV)                                                                                    \
    hipLaunchKernelGGL((backward_kernel<kBackwardQ, QM, NLV>), dim3(n_items), dim3(256), lds, st, kp, items, \
                       elems, groups, img, edof, leaves, V, pt_off, Pt, dLdV, fpart, max_ngrp)
    if (qmode) {
        if (nl == 0) PUFE_BWK(true, 0);
        else if (nl == 2) PUFE_BWK(true, 2);
        else PUFE_BWK(true, 3);
    } else {
        if (nl == 0) PUFE_BWK(false, 0);
        else if (nl == 2) PUFE_BWK(false, 2);
        else PUFE_BWK(false, 3);
    }
#undef PUFE_BWK
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
