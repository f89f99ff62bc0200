// Self-consistent field pieces (section "Self-consistent calculations",
// eqs. poisson and veff): the classical FE space's load vector and evaluation
// at the rule's points, the FE stiffness blocks and the conjugate-gradient
// kernels of the Hartree solve, and the LDA exchange-correlation potential.
#include <hip/hip_runtime.h>

#include "basis.hpp"
#include "device_common.hpp"
#include "scf.hpp"

namespace pufe {

namespace {

constexpr int kLoadThreads = 256;
constexpr int kMaxFe = 32;   // classical FE functions of one element
constexpr int kDotBlocks = 256;

// Values of the element's classical FE functions of order P at reference
// point xi (fully unrolled, so that val stays in registers).
template <int P>
__device__ __forceinline__ void fe_values(const double *xi, double *val) {
    if (P == 3) {
#pragma unroll
        for (int a = 0; a < 32; ++a) {
            double d[3];
            serendipity_fn(a, xi, &val[a], d);
        }
        return;
    }
    constexpr int N1 = P == 3 ? 1 : P + 1;
    double L[3][3], D[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lagrange_1d(P, xi[d], L[d], D[d]);
#pragma unroll
    for (int a3 = 0; a3 < N1; ++a3)
#pragma unroll
        for (int a2 = 0; a2 < N1; ++a2)
#pragma unroll
            for (int a1 = 0; a1 < N1; ++a1) val[a1 + N1 * (a2 + N1 * a3)] = L[0][a1] * L[1][a2] * L[2][a3];
}

// Classical FE index v * nfs + slot of local FE function a of element el.
__device__ __forceinline__ int64_t fe_index(const KParams &kp, const ElemDev &el, const int32_t *edof, int a) {
    int c, s;
    local_slot(el, edof, kp.p, a, &c, &s);
    int j[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        j[d] = el.ijk[d] + ((c >> d) & 1);
        if (j[d] == kp.mesh[d]) j[d] = 0;
    }
    const int64_t v = ((int64_t)j[2] * kp.mesh[1] + j[1]) * kp.mesh[0] + j[0];
    return v * kp.nfs + s;
}

}  // namespace

// be[e][a] = sum over the element's points of w_q phi_a(x_q) f_q: one work
// group per element, per-thread sums over a strided share of the points,
// then a fixed-order tree within each wave and the four wave sums in order
// (deterministic).
template <int P>
__global__ __launch_bounds__(kLoadThreads) void fe_load_elem_kernel(const KParams kp, const ElemDev *__restrict__ elems,
                                                                    const uint32_t *__restrict__ leaves,
                                                                    const double *__restrict__ f,
                                                                    double *__restrict__ be) {
    __shared__ double sW[kLoadThreads / 64][kMaxFe];
    const ElemDev &el = elems[blockIdx.x];
    const int nfe = el.nfe, n3 = kp.n3;
    double acc[kMaxFe];
#pragma unroll
    for (int a = 0; a < kMaxFe; ++a) acc[a] = 0.0;
    const int64_t q0 = el.leaf_off * n3, q1 = el.leaf_end * n3;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kLoadThreads) {
        const int64_t lf = q / n3;
        const int j = (int)(q - lf * n3);
        double xi[3], w, val[kMaxFe];
        leaf_point(kp, leaves[lf], j, xi, &w);
        fe_values<P>(xi, val);
        const double wf = w * f[q];
#pragma unroll
        for (int a = 0; a < kMaxFe; ++a)
            if (a < nfe) acc[a] += wf * val[a];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < kMaxFe; ++a) {
        double v = acc[a];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sW[wave][a] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nfe) {
        double t = sW[0][threadIdx.x];
        for (int k = 1; k < kLoadThreads / 64; ++k) t += sW[k][threadIdx.x];
        be[(int64_t)blockIdx.x * kMaxFe + threadIdx.x] = t;
    }
}

// b[v * nfs + s] = sum of be over the (element, local function) pairs of the
// DOF in element order (dof_el lists of the global DOF dof_off[v] + s).
__global__ void fe_gather_kernel(int64_t nv, int nfs, const int64_t *__restrict__ dof_off,
                                 const int64_t *__restrict__ dof_el_off, const int2 *__restrict__ dof_el,
                                 const double *__restrict__ be, double *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv * nfs) return;
    const int64_t v = i / nfs, g = dof_off[v] + (i - v * nfs);
    double acc = 0.0;
    for (int64_t k = dof_el_off[g]; k < dof_el_off[g + 1]; ++k) acc += be[(int64_t)dof_el[k].x * kMaxFe + dof_el[k].y];
    b[i] = acc;
}

// out_q = sum_a u[fe(a)] phi_a(x_q), one thread per point.
template <int P>
__global__ void fe_eval_kernel(const KParams kp, const ElemDev *__restrict__ elems, const int32_t *__restrict__ edof,
                               const uint32_t *__restrict__ leaves, const int32_t *__restrict__ leaf_elem,
                               int64_t n_qp, const double *__restrict__ u, double *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_qp) return;
    const int64_t lf = q / kp.n3;
    const int j = (int)(q - lf * kp.n3);
    const ElemDev &el = elems[leaf_elem[lf]];
    double xi[3], w, val[kMaxFe];
    leaf_point(kp, leaves[lf], j, xi, &w);
    fe_values<P>(xi, val);
    constexpr int NFE = P == 1 ? 8 : (P == 2 ? 27 : 32);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < NFE; ++a) acc += u[fe_index(kp, el, edof, a)] * val[a];
    out[q] = acc;
}

// K[blk][s][t] = scale * A[bval_off[blk] + s * b_w + t] for s, t < nfs: the
// classical FE rows and columns of every BSR block (b_w = width of the block
// column's vertex).
__global__ void fe_blocks_kernel(int64_t nnzb, int nfs, const int32_t *__restrict__ bcol,
                                 const int64_t *__restrict__ bval_off, const int64_t *__restrict__ dof_off,
                                 const double *__restrict__ A, double scale, double *__restrict__ K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nfs * nfs;
    if (i >= nnzb * per) return;
    const int64_t blk = i / per;
    const int s = (int)((i - blk * per) / nfs), t = (int)(i - blk * per - (int64_t)s * nfs);
    const int64_t w = bcol[blk], bw = dof_off[w + 1] - dof_off[w];
    K[i] = scale * A[bval_off[blk] + s * bw + t];
}

// y = K x over the classical FE space (block rows per vertex).
__global__ void fe_spmv_kernel(int64_t nv, int nfs, const int64_t *__restrict__ brow_ptr,
                               const int32_t *__restrict__ bcol, const double *__restrict__ K,
                               const double *__restrict__ x, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv * nfs) return;
    const int64_t v = i / nfs;
    const int s = (int)(i - v * nfs);
    double acc = 0.0;
    for (int64_t k = brow_ptr[v]; k < brow_ptr[v + 1]; ++k) {
        const double *Kb = K + k * nfs * nfs + (int64_t)s * nfs;
        const double *xb = x + (int64_t)bcol[k] * nfs;
        for (int t = 0; t < nfs; ++t) acc += Kb[t] * xb[t];
    }
    y[i] = acc;
}

// Dot product in a fixed order: kDotBlocks partial sums (grid-strided, tree
// per block), then one block sums them.
__global__ __launch_bounds__(256) void dot_partial_kernel(int64_t n, const double *__restrict__ a,
                                                          const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc += a[i] * b[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void dot_final_kernel(int n, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// y = a x + b y
__global__ void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

// y = a (x - c z)
__global__ void scaled_diff_kernel(int64_t n, double a, const double *__restrict__ x, double c,
                                   const double *__restrict__ z, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * (x[i] - c * z[i]);
}

// Local-density exchange-correlation of the unpolarised electron gas at
// density n (bohr^-3): Slater exchange e_x = -(3/4)(3 n / pi)^(1/3), v_x =
// 4/3 e_x, and the Perdew-Zunger (1981) fit of the Ceperley-Alder
// correlation energy in r_s = (3 / (4 pi n))^(1/3) (one form for r_s >= 1,
// another below), with v_c = d(n e_c)/dn; zero for n <= 1e-30.
__global__ void lda_xc_kernel(int64_t n, const double *__restrict__ rho, double *__restrict__ vxc,
                              double *__restrict__ exc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = rho[i];
    if (!(d > 1e-30)) {
        vxc[i] = 0.0;
        if (exc) exc[i] = 0.0;
        return;
    }
    const double rs = cbrt(3.0 / (4.0 * M_PI * d));
    const double ex = -0.75 * cbrt(3.0 * d / M_PI), vx = 4.0 / 3.0 * ex;
    double ec, vc;
    if (rs >= 1.0) {
        const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
        const double sr = sqrt(rs), den = 1.0 + b1 * sr + b2 * rs;
        ec = g / den;
        vc = ec * (1.0 + 7.0 / 6.0 * b1 * sr + 4.0 / 3.0 * b2 * rs) / den;
    } else {
        const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
        const double lr = log(rs);
        ec = A * lr + B + C * rs * lr + D * rs;
        vc = A * lr + (B - A / 3.0) + 2.0 / 3.0 * C * rs * lr + (2.0 * D - C) / 3.0 * rs;
    }
    vxc[i] = vx + vc;
    if (exc) exc[i] = ex + ec;
}

static unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_fe_load(const KParams &kp, const ElemDev *elems, int64_t nel, const uint32_t *leaves,
                          const double *f, double *be, int64_t nv, int nfs, const int64_t *dof_off,
                          const int64_t *dof_el_off, const int2 *dof_el, double *b, hipStream_t st) {
    if (nel > 0) {
        if (kp.p == 1) fe_load_elem_kernel<1><<<(unsigned)nel, kLoadThreads, 0, st>>>(kp, elems, leaves, f, be);
        else if (kp.p == 2) fe_load_elem_kernel<2><<<(unsigned)nel, kLoadThreads, 0, st>>>(kp, elems, leaves, f, be);
        else fe_load_elem_kernel<3><<<(unsigned)nel, kLoadThreads, 0, st>>>(kp, elems, leaves, f, be);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nv * nfs == 0) return e;
    fe_gather_kernel<<<blocks_for(nv * nfs), 256, 0, st>>>(nv, nfs, dof_off, dof_el_off, dof_el, be, b);
    return hipGetLastError();
}

hipError_t launch_fe_eval(const KParams &kp, const ElemDev *elems, const int32_t *edof, const uint32_t *leaves,
                          const int32_t *leaf_elem, int64_t n_qp, const double *u, double *out, hipStream_t st) {
    if (n_qp <= 0) return hipSuccess;
    if (kp.p == 1) fe_eval_kernel<1><<<blocks_for(n_qp), 256, 0, st>>>(kp, elems, edof, leaves, leaf_elem, n_qp, u, out);
    else if (kp.p == 2) fe_eval_kernel<2><<<blocks_for(n_qp), 256, 0, st>>>(kp, elems, edof, leaves, leaf_elem, n_qp, u, out);
    else fe_eval_kernel<3><<<blocks_for(n_qp), 256, 0, st>>>(kp, elems, edof, leaves, leaf_elem, n_qp, u, out);
    return hipGetLastError();
}

hipError_t launch_fe_blocks(int64_t nnzb, int nfs, const int32_t *bcol, const int64_t *bval_off,
                            const int64_t *dof_off, const double *A, double scale, double *K, hipStream_t st) {
    const int64_t n = nnzb * nfs * nfs;
    if (n <= 0) return hipSuccess;
    fe_blocks_kernel<<<blocks_for(n), 256, 0, st>>>(nnzb, nfs, bcol, bval_off, dof_off, A, scale, K);
    return hipGetLastError();
}

hipError_t launch_fe_spmv(int64_t nv, int nfs, const int64_t *brow_ptr, const int32_t *bcol, const double *K,
                          const double *x, double *y, hipStream_t st) {
    if (nv * nfs <= 0) return hipSuccess;
    fe_spmv_kernel<<<blocks_for(nv * nfs), 256, 0, st>>>(nv, nfs, brow_ptr, bcol, K, x, y);
    return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, hipStream_t st) {
    dot_partial_kernel<<<kDotBlocks, 256, 0, st>>>(n, a, b, part);
    dot_final_kernel<<<1, 256, 0, st>>>(kDotBlocks, part, out);
    return hipGetLastError();
}

int dot_partial_slots() { return kDotBlocks; }

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    axpby_kernel<<<blocks_for(n), 256, 0, st>>>(n, a, x, b, y);
    return hipGetLastError();
}

hipError_t launch_scaled_diff(int64_t n, double a, const double *x, double c, const double *z, double *y,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    scaled_diff_kernel<<<blocks_for(n), 256, 0, st>>>(n, a, x, c, z, y);
    return hipGetLastError();
}

hipError_t launch_lda_xc(int64_t n, const double *rho, double *vxc, double *exc, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    lda_xc_kernel<<<blocks_for(n), 256, 0, st>>>(n, rho, vxc, exc);
    return hipGetLastError();
}

}  // namespace pufe
