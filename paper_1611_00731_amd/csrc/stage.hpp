// Device building blocks shared by the FP64 and split-precision contraction
// kernels: per-point geometry of a work item's stage, the enrichment
// functions of a group, and the unweighted local basis functions (FE, and PU
// times enrichment) with their gradients (eq. pufebasis).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "enrich.hpp"
#include "tables.hpp"

// Global-memory pointer qualifier (address space 1 of the AMDGPU target).
#define PUFE_GLOBAL __attribute__((address_space(1)))

namespace pufe {

// Geometry record of one point (offsets into GEO doubles):
//   xi, x, sqrt(w/2), sqrt(w), 1D FE values L[d][0..2] and derivatives
//   D[d][0..2], trilinear PU values M_c and their 1D factors m_d^0, m_d^1.
enum { G_XI = 0, G_X = 3, G_SW2 = 6, G_SW = 7, G_L = 8, G_D = 17, G_M = 26, G_M1 = 34 };

// Enrichment functions of one group at one point, for groups up to LMAX;
// function m of the group at o[m * FS], component c at o[m * FS + c * Q];
// wimg: image weights (group_eval), null for the periodic enrichment.
template <int LMAX, int Q, int FS = 4 * Q, bool TAB = true>
__device__ __forceinline__ void group_eval_upto(const GroupDev &G, const double *__restrict__ img,
                                                const double *__restrict__ spl, const double *__restrict__ wimg,
                                                const double *x, double *o) {
    switch (G.l) {
        case 0: group_eval<0, FS, Q, TAB>(G, img, spl, wimg, x, o); break;
        case 1: if (LMAX >= 1) group_eval<1, FS, Q, TAB>(G, img, spl, wimg, x, o); break;
        case 2: if (LMAX >= 2) group_eval<2, FS, Q, TAB>(G, img, spl, wimg, x, o); break;
        default: if (LMAX >= 3) group_eval<3, FS, Q, TAB>(G, img, spl, wimg, x, o); break;
    }
}

// The per-launch constants the inner loops use, copied out of KParams into
// registers once per item (KParams of a batched launch lives in global memory).
struct KLocal {
    double E[9], Jt[9], jac, sjac;
    int p, n, n3;
    bool jdiag;   // Jt diagonal (orthogonal cell axes)
    const double *spl;   // tabulated radial coefficients
    const double *wimg;  // image weights of a Bloch-periodic enrichment (null: periodic)
};

__device__ __forceinline__ KLocal load_klocal(const KParams &kp) {
    KLocal k;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        k.E[i] = kp.E[i];
        k.Jt[i] = kp.Jt[i];
    }
    k.jac = kp.jac;
    k.sjac = sqrt(kp.jac);
    k.jdiag = kp.Jt[1] == 0.0 && kp.Jt[2] == 0.0 && kp.Jt[3] == 0.0 && kp.Jt[5] == 0.0 && kp.Jt[6] == 0.0 &&
              kp.Jt[7] == 0.0;
    k.p = kp.p;
    k.n = kp.n;
    k.n3 = kp.n3;
    k.spl = kp.spl;
    k.wimg = kp.wimg;
    return k;
}

// Reference coordinates of point li of the item and the square root of its
// weight, sw = sqrt(w); sGs holds the square roots of the 1D Gauss weights,
// so that sw = h^(3/2) sqrt(det J) prod_d sqrt(w_d) needs no square root per
// point (sw = 0 past the end).
__device__ __forceinline__ void item_point(const KLocal &kp, const uint32_t *sLeaf, const uint32_t *sPt,
                                           const double *sGx, const double *sGs, uint32_t li, uint32_t nli,
                                           uint32_t n3, double *xi, double *sw) {
    xi[0] = xi[1] = xi[2] = 0.0;
    *sw = 0.0;
    if (li >= nli) return;
    const uint32_t lf = li / n3, j = li - lf * n3;
    const uint32_t code = sLeaf[lf], pt = sPt[j];
    const int lev = (int)(code >> 27);
    const double h = 1.0 / (double)(1u << lev);
    const int c[3] = {(int)(code & 511u), (int)((code >> 9) & 511u), (int)((code >> 18) & 511u)};
    const int k[3] = {(int)(pt & 255u), (int)((pt >> 8) & 255u), (int)(pt >> 16)};
    // h^(3/2) = 2^(-3 lev / 2)
    double s = ldexp((lev & 1) ? M_SQRT2 : 1.0, -((3 * lev + (lev & 1)) >> 1)) * kp.sjac;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xi[d] = -1.0 + (2.0 * c[d] + 1.0 + sGx[k[d]]) * h;
        s *= sGs[k[d]];
    }
    *sw = s;
}

__device__ __forceinline__ void point_position(const KLocal &kp, const double *org, const double *xi, double *x) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
        x[cc] = org[cc] + 0.5 * (xi[0] + 1.0) * kp.E[cc] + 0.5 * (xi[1] + 1.0) * kp.E[3 + cc] +
                0.5 * (xi[2] + 1.0) * kp.E[6 + cc];
}

// Geometry record of one point, field f at g[f * Q].
template <int Q>
__device__ __forceinline__ void point_geometry(const KLocal &kp, const double *org, const double *xi, double sw,
                                               double *g) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g[(G_XI + d) * Q] = xi[d];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
        g[(G_X + cc) * Q] = org[cc] + 0.5 * (xi[0] + 1.0) * kp.E[cc] + 0.5 * (xi[1] + 1.0) * kp.E[3 + cc] +
                            0.5 * (xi[2] + 1.0) * kp.E[6 + cc];
    g[G_SW2 * Q] = M_SQRT1_2 * sw;
    g[G_SW * Q] = sw;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double t = xi[d];
        if (kp.p == 1) {
            g[(G_L + 3 * d) * Q] = 0.5 * (1.0 - t);
            g[(G_L + 3 * d + 1) * Q] = 0.5 * (1.0 + t);
            g[(G_D + 3 * d) * Q] = -0.5;
            g[(G_D + 3 * d + 1) * Q] = 0.5;
        } else {
            g[(G_L + 3 * d) * Q] = 0.5 * t * (t - 1.0);
            g[(G_L + 3 * d + 1) * Q] = 1.0 - t * t;
            g[(G_L + 3 * d + 2) * Q] = 0.5 * t * (t + 1.0);
            g[(G_D + 3 * d) * Q] = t - 0.5;
            g[(G_D + 3 * d + 1) * Q] = -2.0 * t;
            g[(G_D + 3 * d + 2) * Q] = t + 0.5;
        }
        g[(G_M1 + 2 * d) * Q] = 0.5 * (1.0 - t);
        g[(G_M1 + 2 * d + 1) * Q] = 0.5 * (1.0 + t);
    }
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8)
        g[(G_M + c8) * Q] = (0.5 + ((c8 & 1) ? 0.5 : -0.5) * xi[0]) * (0.5 + ((c8 & 2) ? 0.5 : -0.5) * xi[1]) *
                            (0.5 + ((c8 & 4) ? 0.5 : -0.5) * xi[2]);
}

// Value and gradient (physical coordinates) of local function a at the point
// whose geometry record starts at g (field f at g[f * Q]); ps points to the
// element's enrichment table at that point (function f, component c at
// ps[(4 f + c) * Q]).  a < 0 (padding row) gives zeros.
template <int Q, bool GEN = true>
__device__ __forceinline__ void local_row(const KLocal &kp, const double *g, const double *ps, const int32_t *sEd,
                                          int a, int nfe, double *val, double *gx) {
    *val = 0.0;
    gx[0] = gx[1] = gx[2] = 0.0;
    if (a < 0) return;
    if (GEN && a < nfe && kp.p == 3) {
        const double xi[3] = {g[G_XI * Q], g[(G_XI + 1) * Q], g[(G_XI + 2) * Q]};
        double dxi[3];
        serendipity_fn(a, xi, val, dxi);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            gx[cc] = kp.Jt[3 * cc] * dxi[0] + kp.Jt[3 * cc + 1] * dxi[1] + kp.Jt[3 * cc + 2] * dxi[2];
        return;
    }
    if (a < nfe) {
        int a1, a2, a3;
        if (kp.p == 2) {
            a1 = a % 3;
            a2 = (a / 3) % 3;
            a3 = a / 9;
        } else {
            a1 = a & 1;
            a2 = (a >> 1) & 1;
            a3 = a >> 2;
        }
        const double l1 = g[(G_L + a1) * Q], l2 = g[(G_L + 3 + a2) * Q], l3 = g[(G_L + 6 + a3) * Q];
        *val = l1 * l2 * l3;
        const double dxi[3] = {g[(G_D + a1) * Q] * l2 * l3, l1 * g[(G_D + 3 + a2) * Q] * l3,
                               l1 * l2 * g[(G_D + 6 + a3) * Q]};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            gx[cc] = kp.Jt[3 * cc] * dxi[0] + kp.Jt[3 * cc + 1] * dxi[1] + kp.Jt[3 * cc + 2] * dxi[2];
        return;
    }
    // PU corner c (trilinear) times enrichment function f
    const int pk = sEd[a - nfe];
    const int c = pk & 7, f = (pk >> 3) & 255;
    const int b0 = c & 1, b1 = (c >> 1) & 1, b2 = c >> 2;
    const double m0 = g[(G_M1 + b0) * Q], m1 = g[(G_M1 + 2 + b1) * Q], m2 = g[(G_M1 + 4 + b2) * Q];
    const double M = g[(G_M + c) * Q];
    const double *pf = ps + (size_t)f * 4 * Q;
    const double p0 = pf[0], p1 = pf[Q], p2 = pf[2 * Q], p3 = pf[3 * Q];
    const double dM[3] = {(b0 ? 0.5 : -0.5) * m1 * m2, m0 * (b1 ? 0.5 : -0.5) * m2, m0 * m1 * (b2 ? 0.5 : -0.5)};
    *val = M * p0;
    // grad(M Psi) = Psi grad M + M grad Psi, grad M via Jt
    gx[0] = (kp.Jt[0] * dM[0] + kp.Jt[1] * dM[1] + kp.Jt[2] * dM[2]) * p0 + M * p1;
    gx[1] = (kp.Jt[3] * dM[0] + kp.Jt[4] * dM[1] + kp.Jt[5] * dM[2]) * p0 + M * p2;
    gx[2] = (kp.Jt[6] * dM[0] + kp.Jt[7] * dM[1] + kp.Jt[8] * dM[2]) * p0 + M * p3;
}

// Rows of whole elements, grouped so that one thread reuses the geometry of
// its point over several rows.  out(a, x, y, z, u) receives, for local
// function a, sqrt(w/2) grad phi_a (x, y, z) and sqrt(w) phi_a (u); with
// MASKED the rows are unweighted, grad phi_a and phi_a, and zero where field
// 6 of the geometry record (the weight, in that layout) is zero.
template <int Q, bool MASKED>
__device__ __forceinline__ void row_weights(const double *g, double *s2, double *sw) {
    if (MASKED) {
        *s2 = *sw = g[6 * Q] != 0.0 ? 1.0 : 0.0;
    } else {
        *s2 = g[G_SW2 * Q];
        *sw = g[G_SW * Q];
    }
}

// fe_unit: the N1 FE functions a = a1 + N1 a2 + N1^2 a3, a1 = 0 .. N1 - 1
// (N1 = p + 1 nodes per direction), of one (a2, a3).
template <int Q, int N1, bool MASKED = false, class Out>
__device__ __forceinline__ void fe_unit(const KLocal &kp, const double *g, int a2, int a3, Out &&out) {
    double s2, sw;
    row_weights<Q, MASKED>(g, &s2, &sw);
    const double L2 = g[(G_L + 3 + a2) * Q], D2 = g[(G_D + 3 + a2) * Q];
    const double L3 = g[(G_L + 6 + a3) * Q], D3 = g[(G_D + 6 + a3) * Q];
    const double p = L2 * L3, pd2 = D2 * L3, pd3 = L2 * D3, pw = sw * p;
    if (kp.jdiag) {   // gradient = diag(Jt) times the reference gradient
        const double p0 = s2 * kp.Jt[0] * p, q1 = s2 * kp.Jt[4] * pd2, q2 = s2 * kp.Jt[8] * pd3;
#pragma unroll
        for (int a1 = 0; a1 < N1; ++a1) {
            const double l1 = g[(G_L + a1) * Q], d1 = g[(G_D + a1) * Q];
            out(a1 + N1 * a2 + N1 * N1 * a3, d1 * p0, l1 * q1, l1 * q2, l1 * pw);
        }
        return;
    }
    double sJ[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) sJ[i] = s2 * kp.Jt[i];
#pragma unroll
    for (int a1 = 0; a1 < N1; ++a1) {
        const double l1 = g[(G_L + a1) * Q], d1 = g[(G_D + a1) * Q];
        const double x0 = d1 * p, x1 = l1 * pd2, x2 = l1 * pd3;
        out(a1 + N1 * a2 + N1 * N1 * a3, sJ[0] * x0 + sJ[1] * x1 + sJ[2] * x2, sJ[3] * x0 + sJ[4] * x1 + sJ[5] * x2,
            sJ[6] * x0 + sJ[7] * x1 + sJ[8] * x2, l1 * pw);
    }
}

// se_unit: FE functions of the 32-node serendipity element sharing one
// point: unit u < 8 the corner u, unit 8 + e the two nodes of edge e.
template <int Q, bool MASKED = false, class Out>
__device__ __forceinline__ void se_unit(const KLocal &kp, const double *g, int u, Out &&out) {
    double s2, sw;
    row_weights<Q, MASKED>(g, &s2, &sw);
    const double xi[3] = {g[G_XI * Q], g[(G_XI + 1) * Q], g[(G_XI + 2) * Q]};
    const int a0 = u < 8 ? u : 8 + 2 * (u - 8), na = u < 8 ? 1 : 2;
    for (int t = 0; t < na; ++t) {
        double v, dxi[3];
        serendipity_fn(a0 + t, xi, &v, dxi);
        double gx[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            gx[cc] = s2 * (kp.Jt[3 * cc] * dxi[0] + kp.Jt[3 * cc + 1] * dxi[1] + kp.Jt[3 * cc + 2] * dxi[2]);
        out(a0 + t, gx[0], gx[1], gx[2], sw * v);
    }
}

// Units of FE functions per point: (p + 1)^2 tensor-product groups for the
// Lagrange elements, 8 corners + 12 edges for the serendipity element.
__device__ __forceinline__ int fe_units(int p) { return p == 3 ? 20 : (p + 1) * (p + 1); }

// FE unit u of any element order (see fe_unit and se_unit); GEN = false
// compiles the Lagrange orders only (kernels of problems of order 1 or 2).
template <int Q, bool MASKED = false, bool GEN = true, class Out>
__device__ __forceinline__ void fe_unit_any(const KLocal &kp, const double *g, int u, Out &&out) {
    if (GEN && kp.p == 3) se_unit<Q, MASKED>(kp, g, u, out);
    else if (kp.p == 2) fe_unit<Q, 3, MASKED>(kp, g, u % 3, u / 3, out);
    else fe_unit<Q, 2, MASKED>(kp, g, u & 1, u >> 1, out);
}

// pu_unit: the enriched functions M_c Psi_f of PU corner c, entries
// kb .. ke - 1 of the element's enriched table (local functions nfe + k);
// ps points to the element's enrichment table at the point (function f,
// component c at ps[FS f + c Q], value and gradient first).
template <int Q, int FS = 4 * Q, bool MASKED = false, class Out>
__device__ __forceinline__ void pu_unit(const KLocal &kp, const double *g, const double *ps, const int32_t *sEd, int c,
                                        int kb, int ke, int nfe, Out &&out) {
    double s2, sw;
    row_weights<Q, MASKED>(g, &s2, &sw);
    const int b0 = c & 1, b1 = (c >> 1) & 1, b2 = c >> 2;
    const double m0 = g[(G_M1 + b0) * Q], m1 = g[(G_M1 + 2 + b1) * Q], m2 = g[(G_M1 + 4 + b2) * Q];
    const double M = g[(G_M + c) * Q];
    const double dM[3] = {(b0 ? 0.5 : -0.5) * m1 * m2, m0 * (b1 ? 0.5 : -0.5) * m2, m0 * m1 * (b2 ? 0.5 : -0.5)};
    // grad(M Psi) = Psi grad M + M grad Psi, grad M via Jt
    double jm[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
        jm[cc] = s2 * (kp.Jt[3 * cc] * dM[0] + kp.Jt[3 * cc + 1] * dM[1] + kp.Jt[3 * cc + 2] * dM[2]);
    const double sM = s2 * M, wM = sw * M;
    for (int k = kb; k < ke; ++k) {
        const int f = (sEd[k] >> 3) & 255;
        const double *pf = ps + (size_t)f * FS;
        const double p0 = pf[0], p1 = pf[Q], p2 = pf[2 * Q], p3 = pf[3 * Q];
        out(nfe + k, jm[0] * p0 + sM * p1, jm[1] * p0 + sM * p2, jm[2] * p0 + sM * p3, wM * p0);
    }
}

// Start of each PU corner's entries in an element's enriched table, which
// lists them corner by corner: cs[c] .. cs[c + 1] - 1 belong to corner c
// (cs[8] = number of entries).  Cooperative over the work group; ne =
// number of entries, ed = the table in global memory.
__device__ __forceinline__ void corner_starts(const PUFE_GLOBAL int32_t *ed, int ne, int *cs, int tid, int nt) {
    for (int k = tid; k <= ne; k += nt) {
        const int ck = k < ne ? (ed[k] & 7) : 8;
        const int cp = k > 0 ? (ed[k - 1] & 7) : -1;
        for (int c = cp + 1; c <= ck; ++c) cs[c] = k;
    }
}

// Chunks of the enriched rows of a partial work item (rows [lo0, hi0) and
// [lo1, hi1) of the element's local functions): runs of one PU corner's
// entries, cut to about nt / q rows' worth of (chunk, point) units so that a
// stage's units fill the work group once; packed as corner | first entry << 3
// | end entry << 13.  cs: corner starts (corner_starts); nfu: FE units of the
// item, which take the first units of a pass (-1: no one-pass widening).
// One thread.
__device__ __forceinline__ void row_chunks(const int *cs, int nfe, int lo0, int hi0, int lo1, int hi1, int q, int nt,
                                           int nfu, int *chunk, int *count) {
    const int e0 = max(lo0 - nfe, 0), e1 = max(hi0 - nfe, 0), f0 = max(lo1 - nfe, 0), f1 = max(hi1 - nfe, 0);
    const int total = (e1 - e0) + (f1 - f0);
    // rows per chunk: the item's (row, point) work spread over one pass of
    // the work group, at least 4 rows, and few enough chunks for the table
    int ch = (total * q + nt - 1) / nt;
    ch = max(ch, max(4, (total + kMaxRowChunks - 17) / (kMaxRowChunks - 16)));
    // The runs are cut per PU corner, so these chunks can overflow one pass
    // (nt / q units, nfu of them the FE units) by a few: a second pass then
    // doubles the stage's row time for a handful of units.  With nfu >= 0,
    // longer chunks, up to twice as long, that fit one pass are taken
    // instead (nfu < 0 keeps the chunks as cut).
    auto chunks_of = [&](int len) {
        int m = 0;
        for (int r = 0; r < 2; ++r) {
            const int b = r ? f0 : e0, e = r ? f1 : e1;
            for (int c = 0; c < 8; ++c) m += (max(min(cs[c + 1], e) - max(cs[c], b), 0) + len - 1) / len;
        }
        return m;
    };
    const int room = min(nt / q - nfu, kMaxRowChunks);
    if (nfu >= 0 && total > 0 && room > 0 && chunks_of(ch) > room) {
        int c2 = ch + 1;
        while (c2 < 2 * ch && chunks_of(c2) > room) ++c2;
        if (c2 < 2 * ch) ch = c2;
    }
    int n = 0;
    for (int r = 0; r < 2; ++r) {
        const int b = r ? f0 : e0, e = r ? f1 : e1;
        for (int c = 0; c < 8; ++c) {
            int kb = max(cs[c], b);
            const int ke = min(cs[c + 1], e);
            while (kb < ke && n < kMaxRowChunks) {
                const int kn = min(kb + ch, ke);
                chunk[n++] = c | (kb << 3) | (kn << 13);
                kb = kn;
            }
        }
    }
    *count = n;
}

}  // namespace pufe
