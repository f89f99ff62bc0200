// Bloch-periodic enrichment (eq. Psi with f(R) = exp(i k.R)): per-k image
// weights for the contraction, and the scatter that turns the real Gram
// matrix of the real and imaginary rows into complex element matrices.
#include <hip/hip_runtime.h>

#include "bloch.hpp"
#include "device_common.hpp"

namespace pufe {

// w[i] = cos(2 pi kappa.n_i) for the entries of the real-part groups and
// sin(2 pi kappa.n_i) for those of the imaginary-part copies; nk[4 i .. 4 i + 3]
// = (n_i, kind).
__global__ void image_weights_kernel(const int32_t *__restrict__ nk, int64_t n, double k0, double k1, double k2,
                                     double *__restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *e = nk + 4 * i;
    double sn, cs;
    sincos(2.0 * M_PI * (k0 * e[0] + k1 * e[1] + k2 * e[2]), &sn, &cs);
    w[i] = e[3] ? sn : cs;
}

// Entry (x, y) of the H (c = 0) or S (c = 1) Gram matrix of an element's
// rows, from its summed partial tiles (upper tile pairs; a diagonal tile is
// stored whole).
__device__ __forceinline__ double gram(const double *__restrict__ part, int x, int y, int c) {
    const int lo = x < y ? x : y, hi = x < y ? y : x;
    const int I = lo >> 4, J = hi >> 4;
    const int64_t pidx = (int64_t)J * (J + 1) / 2 + I;
    return part[pidx * 512 + c * 256 + (lo & 15) * 16 + (hi & 15)];
}

// One upper tile pair of one element, one k-point.  Rows are the element's
// real rows (FE functions, and the real parts of the enriched functions) and
// the imaginary parts of the enriched functions; each thread owns one pair
// (A, B), A <= B, of real rows and forms, with A' and B' the imaginary
// partners (absent for FE rows),
//   H_e[a][b] = G(A, B) + G(A', B') + i (G(A, B') - G(A', B)),
// i.e. the integral of conj(phi_a) phi_b, and the same for S.  The boundary
// phase conj(p_a) p_b comes from the FE rows only (the PU functions are
// periodic in this form).  It adds the product to (g_a, g_b) and its
// conjugate to (g_b, g_a).  Elements of one launch share no vertex.
__global__ __launch_bounds__(256) void scatter_bloch_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                            const int2 *__restrict__ list,
                                                            const int32_t *__restrict__ edof,
                                                            const int32_t *__restrict__ bpart,
                                                            const double *__restrict__ partial,
                                                            const double2 *__restrict__ z, int out_dtype,
                                                            void *__restrict__ Hout, void *__restrict__ Sout) {
    const int2 ep = list[blockIdx.x];
    const ElemDev &el = elems[ep.x];
    const int pidx = ep.y, nloc = el.nloc, nfe = el.nfe;
    int J = 0;
    while ((J + 1) * (J + 2) / 2 <= pidx) ++J;
    const int I = pidx - J * (J + 1) / 2;
    const int A = 16 * I + (int)(threadIdx.x >> 4), B = 16 * J + (int)(threadIdx.x & 15);
    if (A >= nloc || B >= nloc || A > B) return;
    const int pa = A < nfe ? -2 : bpart[el.edof_off + (A - nfe)];
    const int pb = B < nfe ? -2 : bpart[el.edof_off + (B - nfe)];
    if (pa == -1 || pb == -1) return;   // an imaginary row
    const int Ai = pa >= 0 ? nfe + pa : -1, Bi = pb >= 0 ? nfe + pb : -1;
    const double *part = partial + el.part_base * 512;   // the K-chunk sums
    double h[2], s[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double re = gram(part, A, B, c), im = 0.0;
        if (Ai >= 0 && Bi >= 0) re += gram(part, Ai, Bi, c);
        if (Bi >= 0) im += gram(part, A, Bi, c);
        if (Ai >= 0) im -= gram(part, Ai, B, c);
        (c ? s : h)[0] = re;
        (c ? s : h)[1] = im;
    }
    int ca, sa, cb, sb;
    local_slot(el, edof, kp.p, A, &ca, &sa);
    local_slot(el, edof, kp.p, B, &cb, &sb);
    const int64_t oab = el.blk[ca * 8 + cb] + (int64_t)sa * el.bw[cb] + sb;
    const int64_t oba = el.blk[cb * 8 + ca] + (int64_t)sb * el.bw[ca] + sa;
    int t = 0;
    for (int d = 2; d >= 0; --d) {
        const int na = A < nfe ? (el.shifts >> (3 * ca + d)) & 1 : 0;
        const int nb = B < nfe ? (el.shifts >> (3 * cb + d)) & 1 : 0;
        t = 3 * t + (nb - na + 1);
    }
    const double cr = z[t].x, ci = z[t].y;
    const double vh[2] = {cr * h[0] - ci * h[1], cr * h[1] + ci * h[0]};
    const double vs[2] = {cr * s[0] - ci * s[1], cr * s[1] + ci * s[0]};
    if (out_dtype == 0) {
        double *H = (double *)Hout, *S = (double *)Sout;
        H[2 * oab] += vh[0];
        H[2 * oab + 1] += vh[1];
        if (A != B) {
            H[2 * oba] += vh[0];
            H[2 * oba + 1] -= vh[1];
        }
        if (S) {
            S[2 * oab] += vs[0];
            S[2 * oab + 1] += vs[1];
            if (A != B) {
                S[2 * oba] += vs[0];
                S[2 * oba + 1] -= vs[1];
            }
        }
    } else if (out_dtype == 1) {
        float *H = (float *)Hout, *S = (float *)Sout;
        H[2 * oab] += (float)vh[0];
        H[2 * oab + 1] += (float)vh[1];
        if (A != B) {
            H[2 * oba] += (float)vh[0];
            H[2 * oba + 1] -= (float)vh[1];
        }
        if (S) {
            S[2 * oab] += (float)vs[0];
            S[2 * oab + 1] += (float)vs[1];
            if (A != B) {
                S[2 * oba] += (float)vs[0];
                S[2 * oba + 1] -= (float)vs[1];
            }
        }
    } else {   // real output (Gamma: the imaginary parts vanish)
        double *H = (double *)Hout, *S = (double *)Sout;
        H[oab] += vh[0];
        if (A != B) H[oba] += vh[0];
        if (S) {
            S[oab] += vs[0];
            if (A != B) S[oba] += vs[0];
        }
    }
}

hipError_t launch_image_weights(const int32_t *img_nk, int64_t n, const double kap[3], double *w, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    image_weights_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(img_nk, n, kap[0], kap[1], kap[2], w);
    return hipGetLastError();
}

hipError_t launch_scatter_bloch(const KParams &kp, const ElemDev *elems, const int2 *list, int n,
                                const int32_t *edof, const int32_t *bpart, const double *partial, const double2 *z,
                                int out_dtype, void *H, void *S, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    scatter_bloch_kernel<<<n, 256, 0, st>>>(kp, elems, list, edof, bpart, partial, z, out_dtype, H, S);
    return hipGetLastError();
}

}  // namespace pufe
