/*
 * PUFE assembly oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain FP64, single thread, no BLAS, no blocking or reordering beyond what
 * the definitions state.  Every function names the passage of the paper it
 * follows.  Where the paper leaves a choice open, the reading taken is stated
 * at the function (the same list is kept with the design notes).
 *
 * Readings used throughout:
 *  - formulation with Bloch phase factors on the FE and PU functions and
 *    periodic enrichment functions (f(R) = 1 in eq. Psi), so every element
 *    matrix is real and the k-point enters only through the boundary phases
 *    (section "Self-consistent calculations", cubic FE + trilinear PU);
 *    the Bloch-periodic enrichment (f(R) = exp(i k.R)) goes with periodic PU
 *    functions, and its element matrices are complex and per k-point
 *    (the *_bloch functions);
 *  - k-points in reduced coordinates kappa: a local node whose vertex index
 *    wraps by the lattice shift n carries the phase exp(2 pi i kappa.n);
 *  - the conjugated index of H_ij and S_ij is the row index i (eq. disceig3d);
 *  - real, orthonormal spherical harmonics without the Condon-Shortley phase,
 *    written as solid harmonics r^l Y_lm;
 *  - radial functions r^l exp(-a r^2) (1 - (r/rc)^2)^3 for r < rc, 0 beyond,
 *    or r^l times a cubic spline through tabulated samples times the C^3
 *    cutoff of section "Partition of unity enrichment functions",
 *    unnormalised;
 *  - a vertex carries all 2l+1 functions of a descriptor of atom A iff its
 *    minimum-image distance to A is strictly below the support radius re;
 *  - PU functions live on the vertices only (trilinear, any FE order);
 *  - vertex-major DOF order: FE slots of a vertex, then its enriched functions
 *    ordered by atom, descriptor, m = -l..l.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

struct or_state {
    double lat[9];      /* rows a_d */
    double inv[9];      /* inverse of the row matrix: column d is the dual a*_d */
    double detA;
    int mesh[3], p, nfs, n_atoms, n_enr;
    double *pos;
    int *species;
    int *enr_species, *enr_l;
    double *enr_a, *enr_rc, *enr_re;
    int *enr_nrad;      /* samples of a tabulated radial, 0 = analytic */
    double **enr_u;     /* tabulated: spline knot values u_j */
    double **enr_M;     /* tabulated: spline second derivatives at the knots */
    int q_n, q_nref, q_levels, q_mode;
    double q_dist, q_tol;
    int64_t nel, nv, ndof, nqp, nleaves;
    int64_t *vf_off;    /* nv+1 */
    int *vf;            /* 3 per function: atom, desc, m (m in -l..l) */
    int64_t *dof_off;   /* nv+1 */
    int64_t *leaf_off;  /* nel+1 */
    int *leaf_level, *leaf_ijk;
    int64_t *qp_off;    /* nel+1 */
    double *gx, *gw;    /* Gauss-Legendre rule of order q_n */
};

/* ---------------------------------------------------------------- helpers */

static void inv3(const double *m, double *o, double *det) {
    double d = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6])
             + m[2] * (m[3] * m[7] - m[4] * m[6]);
    *det = d;
    o[0] = (m[4] * m[8] - m[5] * m[7]) / d;
    o[1] = (m[2] * m[7] - m[1] * m[8]) / d;
    o[2] = (m[1] * m[5] - m[2] * m[4]) / d;
    o[3] = (m[5] * m[6] - m[3] * m[8]) / d;
    o[4] = (m[0] * m[8] - m[2] * m[6]) / d;
    o[5] = (m[2] * m[3] - m[0] * m[5]) / d;
    o[6] = (m[3] * m[7] - m[4] * m[6]) / d;
    o[7] = (m[1] * m[6] - m[0] * m[7]) / d;
    o[8] = (m[0] * m[4] - m[1] * m[3]) / d;
}

/* Cartesian vector with reduced coordinates u: sum_d u_d a_d */
static void red2cart(const or_state *s, const double *u, double *x) {
    for (int c = 0; c < 3; ++c)
        x[c] = u[0] * s->lat[0 * 3 + c] + u[1] * s->lat[1 * 3 + c] + u[2] * s->lat[2 * 3 + c];
}

/* reduced coordinates u_d = a*_d . x */
static void cart2red(const or_state *s, const double *x, double *u) {
    for (int d = 0; d < 3; ++d)
        u[d] = x[0] * s->inv[0 * 3 + d] + x[1] * s->inv[1 * 3 + d] + x[2] * s->inv[2 * 3 + d];
}

static double dual_norm(const or_state *s, int d) {
    return sqrt(s->inv[0 * 3 + d] * s->inv[0 * 3 + d] + s->inv[1 * 3 + d] * s->inv[1 * 3 + d]
                + s->inv[2 * 3 + d] * s->inv[2 * 3 + d]);
}

/* integer lattice shifts n_d that can bring tau + n.a within radius R of some
 * point whose reduced coordinates lie in [ulo_d, uhi_d] */
static void image_range(const or_state *s, const double *tau, const double *ulo,
                        const double *uhi, double R, int *lo, int *hi) {
    double t[3];
    cart2red(s, tau, t);
    for (int d = 0; d < 3; ++d) {
        double rad = R * dual_norm(s, d);
        lo[d] = (int)floor(ulo[d] - t[d] - rad) - 1;
        hi[d] = (int)ceil(uhi[d] - t[d] + rad) + 1;
    }
}

/* -------------------------------------------- 1D rules and shape functions */

/* Gauss-Legendre nodes (ascending) and weights on [-1,1]: Newton iteration on
 * the Legendre polynomial P_n, weights 2 / ((1 - x^2) P_n'(x)^2).  The paper
 * integrates with tensor-product Gauss rules on hexahedra (section "Adaptive
 * quadrature"). */
void or_gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Lagrange polynomial j of order p on the equispaced nodes -1 + 2k/p of
 * [-1,1], and its derivative (the classical C0 finite element basis). */
void or_lagrange(int p, int j, double t, double *val, double *der) {
    double nodes[8];
    for (int k = 0; k <= p; ++k) nodes[k] = -1.0 + 2.0 * k / p;
    double v = 1.0;
    for (int m = 0; m <= p; ++m)
        if (m != j) v *= (t - nodes[m]) / (nodes[j] - nodes[m]);
    double dsum = 0.0;
    for (int k = 0; k <= p; ++k) {
        if (k == j) continue;
        double prod = 1.0 / (nodes[j] - nodes[k]);
        for (int m = 0; m <= p; ++m)
            if (m != j && m != k) prod *= (t - nodes[m]) / (nodes[j] - nodes[m]);
        dsum += prod;
    }
    *val = v;
    *der = dsum;
}

/* ------------------------------------------------------ solid harmonics */

/* Real solid harmonics r^l Y_lm (l <= 3) as polynomials: each entry holds a
 * coefficient and the exponents of x, y, z.  Orthonormal on the unit sphere,
 * no Condon-Shortley phase, m = -l..l (eq. Psitilde with real Y_lm). */
typedef struct { double c; int i, j, k; } mono;
typedef struct { int n; mono t[4]; } poly;

static poly solid_poly(int l, int m) {
    poly P;
    memset(&P, 0, sizeof P);
    double k0 = 0.5 * sqrt(1.0 / OR_PI);
    double k1 = sqrt(3.0 / (4.0 * OR_PI));
    double k2a = 0.5 * sqrt(15.0 / OR_PI), k2b = 0.25 * sqrt(5.0 / OR_PI),
           k2c = 0.25 * sqrt(15.0 / OR_PI);
    double k3a = 0.25 * sqrt(35.0 / (2.0 * OR_PI)), k3b = 0.5 * sqrt(105.0 / OR_PI),
           k3c = 0.25 * sqrt(21.0 / (2.0 * OR_PI)), k3d = 0.25 * sqrt(7.0 / OR_PI),
           k3e = 0.25 * sqrt(105.0 / OR_PI);
#define T(cc, a, b, d) P.t[P.n++] = (mono){(cc), (a), (b), (d)}
    if (l == 0) {
        T(k0, 0, 0, 0);
    } else if (l == 1) {
        if (m == -1) T(k1, 0, 1, 0);
        if (m == 0) T(k1, 0, 0, 1);
        if (m == 1) T(k1, 1, 0, 0);
    } else if (l == 2) {
        if (m == -2) T(k2a, 1, 1, 0);
        if (m == -1) T(k2a, 0, 1, 1);
        if (m == 0) { T(2 * k2b, 0, 0, 2); T(-k2b, 2, 0, 0); T(-k2b, 0, 2, 0); }
        if (m == 1) T(k2a, 1, 0, 1);
        if (m == 2) { T(k2c, 2, 0, 0); T(-k2c, 0, 2, 0); }
    } else if (l == 3) {
        if (m == -3) { T(3 * k3a, 2, 1, 0); T(-k3a, 0, 3, 0); }
        if (m == -2) T(k3b, 1, 1, 1);
        if (m == -1) { T(4 * k3c, 0, 1, 2); T(-k3c, 2, 1, 0); T(-k3c, 0, 3, 0); }
        if (m == 0) { T(2 * k3d, 0, 0, 3); T(-3 * k3d, 2, 0, 1); T(-3 * k3d, 0, 2, 1); }
        if (m == 1) { T(4 * k3c, 1, 0, 2); T(-k3c, 3, 0, 0); T(-k3c, 1, 2, 0); }
        if (m == 2) { T(k3e, 2, 0, 1); T(-k3e, 0, 2, 1); }
        if (m == 3) { T(k3a, 3, 0, 0); T(-3 * k3a, 1, 2, 0); }
    }
#undef T
    return P;
}

static double ipow(double x, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

/* x^i with derivative order d: i (i-1) .. x^(i-d), zero when d > i */
static double dpow(double x, int i, int d) {
    if (d > i) return 0.0;
    double c = 1.0;
    for (int k = 0; k < d; ++k) c *= (double)(i - k);
    return c * ipow(x, i - d);
}

void or_solid_harmonic(int l, int m, const double *r, double *val, double *grad, double *hess) {
    poly P = solid_poly(l, m);
    double v = 0.0, g[3] = {0, 0, 0}, h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < P.n; ++t) {
        int e[3] = {P.t[t].i, P.t[t].j, P.t[t].k};
        double c = P.t[t].c;
        v += c * dpow(r[0], e[0], 0) * dpow(r[1], e[1], 0) * dpow(r[2], e[2], 0);
        for (int a = 0; a < 3; ++a) {
            int da[3] = {0, 0, 0};
            da[a] = 1;
            g[a] += c * dpow(r[0], e[0], da[0]) * dpow(r[1], e[1], da[1]) * dpow(r[2], e[2], da[2]);
            for (int b = 0; b < 3; ++b) {
                int db[3] = {da[0], da[1], da[2]};
                db[b] += 1;
                h[a * 3 + b] += c * dpow(r[0], e[0], db[0]) * dpow(r[1], e[1], db[1])
                              * dpow(r[2], e[2], db[2]);
            }
        }
    }
    if (val) *val = v;
    if (grad) memcpy(grad, g, sizeof g);
    if (hess) memcpy(hess, h, sizeof h);
}

/* ------------------------------------------------- enrichment functions */

/* The C^3 cutoff function of section "Partition of unity enrichment
 * functions": h(r, rc) = 1 + 20 x^7 - 70 x^6 + 84 x^5 - 35 x^4 with
 * x = r/rc for r <= rc, and 0 beyond. */
static double cutoff_c3(double r, double rc) {
    if (r >= rc) return 0.0;
    double x = r / rc, x2 = x * x, x4 = x2 * x2;
    return 1.0 + 20.0 * x4 * x2 * x - 70.0 * x4 * x2 + 84.0 * x4 * x - 35.0 * x4;
}

/* Tabulated radial (section "Partition of unity enrichment functions"): the
 * radial R(r) is the cubic spline fit of the pseudoatomic radial times the
 * C^3 cutoff.  The samples t_j are the pseudoatomic radial divided by r^l at
 * r_j = j rc/(n-1); the spline u interpolates u_j = t_j h(r_j, rc) with end
 * slopes u'(0) = 0 (the radial over r^l is even) and u'(rc) = 0 (h vanishes
 * to third order there), and R(r) = r^l u(r).  Second derivatives M_j from
 * the clamped-spline equations
 *   M_{j-1} + 4 M_j + M_{j+1} = 6 (u_{j+1} - 2 u_j + u_{j-1}) / d^2,
 *   2 M_0 + M_1 = 6 (u_1 - u_0) / d^2,
 *   M_{n-2} + 2 M_{n-1} = -6 (u_{n-1} - u_{n-2}) / d^2,
 * solved by forward elimination and back substitution. */
static void spline_fit(int n, double rc, const double *t, double *u, double *M) {
    double d = rc / (n - 1);
    for (int j = 0; j < n; ++j) u[j] = t[j] * cutoff_c3(j * d, rc);
    double *diag = malloc(sizeof(double) * n), *rhs = malloc(sizeof(double) * n);
    for (int j = 0; j < n; ++j) {
        diag[j] = (j == 0 || j == n - 1) ? 2.0 : 4.0;
        if (j == 0) rhs[j] = 6.0 * (u[1] - u[0]) / (d * d);
        else if (j == n - 1) rhs[j] = -6.0 * (u[n - 1] - u[n - 2]) / (d * d);
        else rhs[j] = 6.0 * (u[j + 1] - 2.0 * u[j] + u[j - 1]) / (d * d);
    }
    /* every off-diagonal entry is 1 */
    for (int j = 1; j < n; ++j) {
        double f = 1.0 / diag[j - 1];
        diag[j] -= f;
        rhs[j] -= f * rhs[j - 1];
    }
    M[n - 1] = rhs[n - 1] / diag[n - 1];
    for (int j = n - 2; j >= 0; --j) M[j] = (rhs[j] - M[j + 1]) / diag[j];
    free(diag);
    free(rhs);
}

/* u, u', u'' of the spline of descriptor k at r (0 at and beyond rc), in the
 * interval form u = A u_j + B u_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) d^2/6
 * with A = (r_{j+1} - r)/d, B = 1 - A. */
static void spline_eval(const or_state *s, int k, double r, double *u, double *u1, double *u2) {
    int n = s->enr_nrad[k];
    double rc = s->enr_rc[k], d = rc / (n - 1);
    if (r >= rc) { *u = *u1 = *u2 = 0.0; return; }
    int j = (int)(r / d);
    if (j > n - 2) j = n - 2;
    const double *uu = s->enr_u[k], *M = s->enr_M[k];
    double B = (r - j * d) / d, A = 1.0 - B;
    *u = A * uu[j] + B * uu[j + 1] + ((A * A * A - A) * M[j] + (B * B * B - B) * M[j + 1]) * d * d / 6.0;
    *u1 = (uu[j + 1] - uu[j]) / d - (3.0 * A * A - 1.0) / 6.0 * d * M[j] + (3.0 * B * B - 1.0) / 6.0 * d * M[j + 1];
    *u2 = A * M[j] + B * M[j + 1];
}

/* One lattice image's term of the enrichment sum (eq. Psitilde):
 * Psi~(r) = radial(|r|) S_lm(r) at the offset r = x - tau - R from the image
 * centre, with its gradient and Hessian; zero at and beyond the cutoff.
 * Analytic radial: g(s) = exp(-a s) (1 - s/rc^2)^3 in s = |r|^2; tabulated:
 * the spline u(|r|) (already times the cutoff h). */
static void image_term(const or_state *s, int desc, int m, const double *r, double *val, double *grad,
                       double *hess) {
    int l = s->enr_l[desc];
    double a = s->enr_a[desc], rc = s->enr_rc[desc];
    double sq = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    *val = 0.0;
    for (int i = 0; i < 3; ++i) grad[i] = 0.0;
    for (int i = 0; i < 9; ++i) hess[i] = 0.0;
    if (sq >= rc * rc) return;
    if (s->enr_nrad[desc] > 0) {
        /* tabulated: Psi~ = u(|r|) S_lm(r), with
         * grad u = u' r_hat and
         * hess u = u'' r_hat r_hat^T + (u'/|r|) (I - r_hat r_hat^T) */
        double rr = sqrt(sq), u, u1, u2;
        spline_eval(s, desc, rr, &u, &u1, &u2);
        double S, dS[3], hS[9], rh[3] = {0, 0, 0}, u1r = u2;   /* u'/|r| -> u''(0) at r = 0 */
        if (rr > 0.0) {
            for (int i = 0; i < 3; ++i) rh[i] = r[i] / rr;
            u1r = u1 / rr;
        }
        or_solid_harmonic(l, m, r, &S, dS, hS);
        *val = u * S;
        for (int i = 0; i < 3; ++i) grad[i] = u1 * rh[i] * S + u * dS[i];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double hu = (u2 - u1r) * rh[i] * rh[j] + (i == j ? u1r : 0.0);
                hess[i * 3 + j] = hu * S + u1 * (rh[i] * dS[j] + dS[i] * rh[j]) + u * hS[i * 3 + j];
            }
        return;
    }
    double e = exp(-a * sq), c = 1.0 - sq / (rc * rc);
    double g = e * c * c * c;
    double g1 = -a * e * c * c * c - 3.0 * e * c * c / (rc * rc);
    double g2 = a * a * e * c * c * c + 6.0 * a * e * c * c / (rc * rc)
              + 6.0 * e * c / (rc * rc * rc * rc);
    double S, dS[3], hS[9];
    or_solid_harmonic(l, m, r, &S, dS, hS);
    *val = g * S;
    for (int i = 0; i < 3; ++i) grad[i] = 2.0 * g1 * r[i] * S + g * dS[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            hess[i * 3 + j] = 4.0 * g2 * r[i] * r[j] * S
                            + 2.0 * g1 * ((i == j ? S : 0.0) + r[i] * dS[j] + dS[i] * r[j])
                            + g * hS[i * 3 + j];
}

/* Periodic enrichment function (eqs. Psitilde and Psi with f(R) = 1):
 * Psi(x) = sum over lattice translations R of Psi~(x - tau - R).  Every image
 * within the cutoff is included (for the paper's cells this is its -2..2
 * range).  Returns value, gradient and Hessian. */
void or_enrichment(const or_state *s, int atom, int desc, int m, const double *x,
                   double *val, double *grad, double *hess) {
    double rc = s->enr_rc[desc];
    const double *tau = s->pos + 3 * atom;
    double ux[3];
    cart2red(s, x, ux);
    int lo[3], hi[3];
    image_range(s, tau, ux, ux, rc, lo, hi);
    double v = 0.0, g3[3] = {0, 0, 0}, h9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int n3 = lo[2]; n3 <= hi[2]; ++n3)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
            for (int n1 = lo[0]; n1 <= hi[0]; ++n1) {
                double nn[3] = {(double)n1, (double)n2, (double)n3}, R[3], r[3];
                red2cart(s, nn, R);
                for (int c = 0; c < 3; ++c) r[c] = x[c] - tau[c] - R[c];
                double tv, tg[3], th[9];
                image_term(s, desc, m, r, &tv, tg, th);
                v += tv;
                for (int i = 0; i < 3; ++i) g3[i] += tg[i];
                for (int i = 0; i < 9; ++i) h9[i] += th[i];
            }
    if (val) *val = v;
    if (grad) memcpy(grad, g3, sizeof g3);
    if (hess) memcpy(hess, h9, sizeof h9);
}

/* Bloch-periodic enrichment function (eq. Psi with f(R) = exp(i k.R)):
 * Psi^k(x) = sum over R = n.a of exp(2 pi i kappa.n) Psi~(x - tau - R), tau
 * the atom position as given (moving the atom by a lattice vector multiplies
 * the function by a constant phase).  val[2] = (Re, Im) of the value,
 * grad[6] = the real parts of the gradient, then the imaginary parts. */
void or_enrichment_bloch(const or_state *s, int atom, int desc, int m, const double *x, const double *kappa,
                         double *val, double *grad) {
    double rc = s->enr_rc[desc];
    const double *tau = s->pos + 3 * atom;
    double ux[3];
    cart2red(s, x, ux);
    int lo[3], hi[3];
    image_range(s, tau, ux, ux, rc, lo, hi);
    for (int i = 0; i < 2; ++i) val[i] = 0.0;
    for (int i = 0; i < 6; ++i) grad[i] = 0.0;
    for (int n3 = lo[2]; n3 <= hi[2]; ++n3)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
            for (int n1 = lo[0]; n1 <= hi[0]; ++n1) {
                double nn[3] = {(double)n1, (double)n2, (double)n3}, R[3], r[3];
                red2cart(s, nn, R);
                for (int c = 0; c < 3; ++c) r[c] = x[c] - tau[c] - R[c];
                double tv, tg[3], th[9];
                image_term(s, desc, m, r, &tv, tg, th);
                double t = 2.0 * OR_PI * (kappa[0] * n1 + kappa[1] * n2 + kappa[2] * n3);
                double cr = cos(t), ci = sin(t);
                val[0] += cr * tv;
                val[1] += ci * tv;
                for (int i = 0; i < 3; ++i) {
                    grad[i] += cr * tg[i];
                    grad[3 + i] += ci * tg[i];
                }
            }
}

/* ----------------------------------------------------------- topology */

static void vertex_ijk(const or_state *s, int64_t v, int *j) {
    j[0] = (int)(v % s->mesh[0]);
    j[1] = (int)((v / s->mesh[0]) % s->mesh[1]);
    j[2] = (int)(v / ((int64_t)s->mesh[0] * s->mesh[1]));
}

static int64_t vertex_id(const or_state *s, const int *j) {
    return ((int64_t)j[2] * s->mesh[1] + j[1]) * s->mesh[0] + j[0];
}

static void element_ijk(const or_state *s, int64_t e, int *i) {
    i[0] = (int)(e % s->mesh[0]);
    i[1] = (int)((e / s->mesh[0]) % s->mesh[1]);
    i[2] = (int)(e / ((int64_t)s->mesh[0] * s->mesh[1]));
}

static void vertex_position(const or_state *s, int64_t v, double *x) {
    int j[3];
    vertex_ijk(s, v, j);
    double u[3] = {(double)j[0] / s->mesh[0], (double)j[1] / s->mesh[1], (double)j[2] / s->mesh[2]};
    red2cart(s, u, x);
}

/* Smallest distance between x and any lattice image of tau. */
static double min_image_distance(const or_state *s, const double *x, const double *tau, double R) {
    double ux[3];
    cart2red(s, x, ux);
    int lo[3], hi[3];
    image_range(s, tau, ux, ux, R, lo, hi);
    double best = INFINITY;
    for (int n3 = lo[2]; n3 <= hi[2]; ++n3)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
            for (int n1 = lo[0]; n1 <= hi[0]; ++n1) {
                double nn[3] = {(double)n1, (double)n2, (double)n3}, Rv[3];
                red2cart(s, nn, Rv);
                double d2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    double t = x[c] - tau[c] - Rv[c];
                    d2 += t * t;
                }
                if (d2 < best) best = d2;
            }
    return sqrt(best);
}

/* Local functions of one element. */
typedef struct {
    int64_t g;      /* global DOF */
    int64_t fe;     /* FE node: index v * nfs + slot in the classical FE space */
    int shift[3];   /* lattice shift of the node's vertex */
    int kind;       /* 0 FE node, 1 enriched */
    int node[3];    /* FE: node index per dimension (0..p; serendipity: 0..3 for -1, -1/3, 1/3, 1) */
    int corner;     /* enriched: corner c = c1 + 2 c2 + 4 c3 */
    int atom, desc, m;
} loc_fn;

static int max_locals(const or_state *s) {
    int64_t mx = 0;
    for (int64_t v = 0; v < s->nv; ++v)
        if (s->vf_off[v + 1] - s->vf_off[v] > mx) mx = s->vf_off[v + 1] - s->vf_off[v];
    return (s->p == 3 ? 32 : (s->p + 1) * (s->p + 1) * (s->p + 1)) + 8 * (int)mx;
}

/* Element-local ordering: the FE nodes (lexicographic, first index fastest),
 * then the 8 corners c, each with its vertex's enriched functions in vertex
 * order.  A node on the upper face of the cell wraps to vertex index 0 and
 * records the lattice shift 1 in that direction (Bloch-periodic FE and PU,
 * section "Self-consistent calculations"). */
static int element_locals(const or_state *s, int64_t e, loc_fn *L) {
    int i[3], n = 0;
    element_ijk(s, e, i);
    if (s->p == 1 || s->p == 2) {
        int p = s->p;
        for (int a3 = 0; a3 <= p; ++a3)
            for (int a2 = 0; a2 <= p; ++a2)
                for (int a1 = 0; a1 <= p; ++a1) {
                    int a[3] = {a1, a2, a3}, j[3], slot = 0;
                    loc_fn f;
                    memset(&f, 0, sizeof f);
                    for (int d = 0; d < 3; ++d) {
                        int up = (a[d] == p) ? 1 : 0;   /* node sits on the next vertex */
                        int mid = (p == 2 && a[d] == 1) ? 1 : 0;
                        j[d] = i[d] + up;
                        f.shift[d] = 0;
                        if (j[d] >= s->mesh[d]) { j[d] -= s->mesh[d]; f.shift[d] = 1; }
                        slot += mid << d;
                        f.node[d] = a[d];
                    }
                    f.kind = 0;
                    f.g = s->dof_off[vertex_id(s, j)] + slot;
                    f.fe = vertex_id(s, j) * s->nfs + slot;
                    L[n++] = f;
                }
    } else { /* 32-node serendipity topology: corners, then 2 nodes per edge */
        for (int c = 0; c < 8; ++c) {
            int j[3];
            loc_fn f;
            memset(&f, 0, sizeof f);
            for (int d = 0; d < 3; ++d) {
                j[d] = i[d] + ((c >> d) & 1);
                if (j[d] >= s->mesh[d]) { j[d] -= s->mesh[d]; f.shift[d] = 1; }
            }
            f.g = s->dof_off[vertex_id(s, j)];
            f.fe = vertex_id(s, j) * s->nfs;
            for (int d = 0; d < 3; ++d) f.node[d] = 3 * ((c >> d) & 1);
            L[n++] = f;
        }
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 8; ++c) {
                if ((c >> d) & 1) continue;   /* edge along d starts at a corner with c_d = 0 */
                int j[3];
                int sh[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) {
                    j[k] = i[k] + ((c >> k) & 1);
                    if (j[k] >= s->mesh[k]) { j[k] -= s->mesh[k]; sh[k] = 1; }
                }
                for (int t = 0; t < 2; ++t) {
                    loc_fn f;
                    memset(&f, 0, sizeof f);
                    memcpy(f.shift, sh, sizeof sh);
                    f.g = s->dof_off[vertex_id(s, j)] + 1 + 2 * d + t;
                    f.fe = vertex_id(s, j) * s->nfs + 1 + 2 * d + t;
                    for (int k = 0; k < 3; ++k) f.node[k] = 3 * ((c >> k) & 1);
                    f.node[d] = 1 + t;   /* the edge nodes at -1/3 and +1/3 */
                    L[n++] = f;
                }
            }
    }
    for (int c = 0; c < 8; ++c) {
        int j[3], sh[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            j[d] = i[d] + ((c >> d) & 1);
            if (j[d] >= s->mesh[d]) { j[d] -= s->mesh[d]; sh[d] = 1; }
        }
        int64_t v = vertex_id(s, j);
        for (int64_t k = s->vf_off[v]; k < s->vf_off[v + 1]; ++k) {
            loc_fn f;
            memset(&f, 0, sizeof f);
            f.kind = 1;
            f.corner = c;
            memcpy(f.shift, sh, sizeof sh);
            f.atom = s->vf[3 * k];
            f.desc = s->vf[3 * k + 1];
            f.m = s->vf[3 * k + 2];
            f.g = s->dof_off[v] + s->nfs + (k - s->vf_off[v]);
            L[n++] = f;
        }
    }
    return n;
}

/* ------------------------------------------------------ basis at a point */

static void element_origin(const or_state *s, int64_t e, double *x0) {
    int i[3];
    element_ijk(s, e, i);
    double u[3] = {(double)i[0] / s->mesh[0], (double)i[1] / s->mesh[1], (double)i[2] / s->mesh[2]};
    red2cart(s, u, x0);
}

/* x(xi) = x0 + sum_d ((xi_d + 1)/2) a_d / n_d */
static void ref2phys(const or_state *s, int64_t e, const double *xi, double *x) {
    double x0[3];
    element_origin(s, e, x0);
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = 0.5 * (xi[d] + 1.0) / s->mesh[d];
    red2cart(s, u, x);
    for (int c = 0; c < 3; ++c) x[c] += x0[c];
}

/* Cartesian gradient from reference derivatives: grad_x = sum_d dphi/dxi_d * 2 n_d a*_d */
static void ref_grad(const or_state *s, const double *dxi, double *g) {
    for (int c = 0; c < 3; ++c) {
        g[c] = 0.0;
        for (int d = 0; d < 3; ++d) g[c] += dxi[d] * 2.0 * s->mesh[d] * s->inv[c * 3 + d];
    }
}

/* 32-node cubic serendipity hexahedron (the paper's classical FE in section
 * "Self-consistent calculations"): nodes at the corners (coordinates +-1) and
 * at +-1/3 along every edge.  With the node at (a, b, c), reference point
 * (x, y, z):
 *   corner:            (1 + a x)(1 + b y)(1 + c z)(9 (x^2 + y^2 + z^2) - 19) / 64,
 *   edge along x:  9 (1 - x^2)(1 + 9 a x)(1 + b y)(1 + c z) / 64,
 * and alike for edges along y and z.  Returns the value and the reference
 * gradient. */
static void serendipity(const int *node, const double *xi, double *val, double *dxi) {
    double nc[3];
    int edge = -1;
    for (int d = 0; d < 3; ++d) {
        nc[d] = -1.0 + 2.0 * node[d] / 3.0;
        if (node[d] == 1 || node[d] == 2) edge = d;
    }
    if (edge < 0) {
        double f[3], r = 9.0 * (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) - 19.0;
        for (int d = 0; d < 3; ++d) f[d] = 1.0 + nc[d] * xi[d];
        *val = f[0] * f[1] * f[2] * r / 64.0;
        for (int d = 0; d < 3; ++d) {
            double other = 1.0;
            for (int k = 0; k < 3; ++k)
                if (k != d) other *= f[k];
            dxi[d] = (nc[d] * other * r + f[0] * f[1] * f[2] * 18.0 * xi[d]) / 64.0;
        }
        return;
    }
    double f[3], df[3];
    for (int d = 0; d < 3; ++d) {
        if (d == edge) {
            double t = xi[d], a = nc[d];
            f[d] = (1.0 - t * t) * (1.0 + 9.0 * a * t);
            df[d] = -2.0 * t * (1.0 + 9.0 * a * t) + (1.0 - t * t) * 9.0 * a;
        } else {
            f[d] = 1.0 + nc[d] * xi[d];
            df[d] = nc[d];
        }
    }
    *val = 9.0 * f[0] * f[1] * f[2] / 64.0;
    dxi[0] = 9.0 * df[0] * f[1] * f[2] / 64.0;
    dxi[1] = 9.0 * f[0] * df[1] * f[2] / 64.0;
    dxi[2] = 9.0 * f[0] * f[1] * df[2] / 64.0;
}

/* Values and gradients of the element's PUFE basis (eq. pufebasis): classical
 * FE functions and PU functions times enrichment functions. */
/* Value and Cartesian gradient of one classical FE function (serendipity,
 * or the tensor product of 1D Lagrange factors). */
static void fe_function(const or_state *s, const loc_fn *f, const double *xi, double *val, double *grad) {
    if (s->p == 3) {
        double dxi[3];
        serendipity(f->node, xi, val, dxi);
        ref_grad(s, dxi, grad);
        return;
    }
    double v = 1.0, dxi[3] = {1.0, 1.0, 1.0};
    for (int d = 0; d < 3; ++d) {
        double lv, ld;
        or_lagrange(s->p, f->node[d], xi[d], &lv, &ld);
        for (int k = 0; k < 3; ++k) dxi[k] *= (k == d) ? ld : lv;
        v *= lv;
    }
    *val = v;
    ref_grad(s, dxi, grad);
}

static void basis_eval(const or_state *s, int64_t e, const loc_fn *L, int nloc, const double *xi,
                       double *val, double *grad) {
    double x[3];
    ref2phys(s, e, xi, x);
    for (int a = 0; a < nloc; ++a) {
        if (L[a].kind == 0) {
            fe_function(s, &L[a], xi, &val[a], grad + 3 * a);
        } else {
            double M = 1.0, dxi[3] = {1.0, 1.0, 1.0};
            for (int d = 0; d < 3; ++d) {
                double lv, ld;
                or_lagrange(1, (L[a].corner >> d) & 1, xi[d], &lv, &ld);
                for (int k = 0; k < 3; ++k) dxi[k] *= (k == d) ? ld : lv;
                M *= lv;
            }
            double gM[3], psi, gpsi[3];
            ref_grad(s, dxi, gM);
            or_enrichment(s, L[a].atom, L[a].desc, L[a].m, x, &psi, gpsi, NULL);
            val[a] = M * psi;
            for (int c = 0; c < 3; ++c) grad[3 * a + c] = gM[c] * psi + M * gpsi[c];
        }
    }
}

void or_basis_at(const or_state *s, int64_t e, const double *xi, double *val, double *grad) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    basis_eval(s, e, L, n, xi, val, grad);
    free(L);
}

/* ------------------------------------------------------------ quadrature */

typedef struct {
    int *level, *ijk;
    int64_t n, cap;
} leaf_list;

static void push_leaf(leaf_list *ll, int lev, const int *c) {
    if (ll->n == ll->cap) {
        ll->cap = ll->cap ? 2 * ll->cap : 1024;
        ll->level = realloc(ll->level, sizeof(int) * ll->cap);
        ll->ijk = realloc(ll->ijk, sizeof(int) * 3 * ll->cap);
    }
    ll->level[ll->n] = lev;
    memcpy(ll->ijk + 3 * ll->n, c, 3 * sizeof(int));
    ll->n++;
}

/* reference interval of cell (lev, c) along one direction */
static void cell_interval(int lev, int c, double *lo, double *hi) {
    double h = 2.0 / (double)(1 << lev);
    *lo = -1.0 + c * h;
    *hi = -1.0 + (c + 1) * h;
}

/* Geometric refinement (the reading taken for the synthetic workloads): a
 * cell is split while its level is below the maximum and the closest point of
 * its (axis-aligned) box lies within q_dist of some nucleus image. */
static int geom_split(const or_state *s, int64_t e, int lev, const int *c) {
    if (lev >= s->q_levels) return 0;
    int i[3];
    element_ijk(s, e, i);
    double blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
        double lo, hi;
        cell_interval(lev, c[d], &lo, &hi);
        double L = s->lat[d * 3 + d];
        blo[d] = (i[d] + 0.5 * (lo + 1.0)) / s->mesh[d] * L;
        bhi[d] = (i[d] + 0.5 * (hi + 1.0)) / s->mesh[d] * L;
    }
    for (int A = 0; A < s->n_atoms; ++A) {
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            double L = s->lat[d * 3 + d], t = s->pos[3 * A + d];
            int mlo = (int)floor((blo[d] - s->q_dist - t) / L) - 1;
            int mhi = (int)ceil((bhi[d] + s->q_dist - t) / L) + 1;
            double best = INFINITY;
            for (int m = mlo; m <= mhi; ++m) {
                double y = t + m * L, dd = 0.0;
                if (y < blo[d]) dd = blo[d] - y;
                else if (y > bhi[d]) dd = y - bhi[d];
                if (dd < best) best = dd;
            }
            d2 += best * best;
        }
        if (sqrt(d2) <= s->q_dist) return 1;
    }
    return 0;
}

static void geom_cell(const or_state *s, int64_t e, int lev, const int *c, leaf_list *ll) {
    if (!geom_split(s, e, lev, c)) {
        push_leaf(ll, lev, c);
        return;
    }
    for (int ch = 0; ch < 8; ++ch) {
        int cc[3] = {2 * c[0] + (ch & 1), 2 * c[1] + ((ch >> 1) & 1), 2 * c[2] + ((ch >> 2) & 1)};
        geom_cell(s, e, lev + 1, cc, ll);
    }
}

/* tensor Gauss rule of order n on cell (lev, c) of element e: integrals of
 * Psi^2 and |grad Psi|^2 for one enrichment function */
static void cell_integrals(const or_state *s, int64_t e, int lev, const int *c, int n,
                           int atom, int desc, int m, double *I0, double *I1) {
    double *x = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    or_gauss_legendre(n, x, w);
    double jac = s->detA / (8.0 * s->mesh[0] * s->mesh[1] * s->mesh[2]);
    double h = 1.0 / (double)(1 << lev);
    double a0 = 0.0, a1 = 0.0;
    for (int k3 = 0; k3 < n; ++k3)
        for (int k2 = 0; k2 < n; ++k2)
            for (int k1 = 0; k1 < n; ++k1) {
                int kk[3] = {k1, k2, k3};
                double xi[3], X[3];
                for (int d = 0; d < 3; ++d) {
                    double lo, hi;
                    cell_interval(lev, c[d], &lo, &hi);
                    xi[d] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * x[kk[d]];
                }
                ref2phys(s, e, xi, X);
                double wt = w[k1] * w[k2] * w[k3] * h * h * h * jac, psi, g[3];
                or_enrichment(s, atom, desc, m, X, &psi, g, NULL);
                a0 += wt * psi * psi;
                a1 += wt * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            }
    free(x);
    free(w);
    *I0 = a0;
    *I1 = a1;
}

/* Error-driven refinement (section "Adaptive quadrature"): every enrichment
 * function still in the active set is integrated as Psi^2 and |grad Psi|^2
 * with the base rule and with the reference rule; a cell is split into 8 when
 * one of them misses the absolute tolerance, and only the functions that
 * missed it are tested on the children. */
static void error_cell(const or_state *s, int64_t e, int lev, const int *c, const int *fns,
                       int nf, leaf_list *ll) {
    int *fail = malloc(sizeof(int) * 3 * (nf > 0 ? nf : 1));
    int nfail = 0;
    if (lev < s->q_levels) {
        for (int f = 0; f < nf; ++f) {
            double b0, b1, r0, r1;
            cell_integrals(s, e, lev, c, s->q_n, fns[3 * f], fns[3 * f + 1], fns[3 * f + 2], &b0, &b1);
            cell_integrals(s, e, lev, c, s->q_nref, fns[3 * f], fns[3 * f + 1], fns[3 * f + 2], &r0, &r1);
            if (fabs(b0 - r0) > s->q_tol || fabs(b1 - r1) > s->q_tol) {
                memcpy(fail + 3 * nfail, fns + 3 * f, 3 * sizeof(int));
                nfail++;
            }
        }
    }
    if (nfail == 0) {
        push_leaf(ll, lev, c);
    } else {
        for (int ch = 0; ch < 8; ++ch) {
            int cc[3] = {2 * c[0] + (ch & 1), 2 * c[1] + ((ch >> 1) & 1), 2 * c[2] + ((ch >> 2) & 1)};
            error_cell(s, e, lev + 1, cc, fail, nfail, ll);
        }
    }
    free(fail);
}

/* enrichment functions carried by at least one corner of element e */
static int element_functions(const or_state *s, int64_t e, int *fns) {
    int i[3], nf = 0;
    element_ijk(s, e, i);
    for (int c = 0; c < 8; ++c) {
        int j[3];
        for (int d = 0; d < 3; ++d) j[d] = (i[d] + ((c >> d) & 1)) % s->mesh[d];
        int64_t v = vertex_id(s, j);
        for (int64_t k = s->vf_off[v]; k < s->vf_off[v + 1]; ++k) {
            int dup = 0;
            for (int f = 0; f < nf; ++f)
                if (fns[3 * f] == s->vf[3 * k] && fns[3 * f + 1] == s->vf[3 * k + 1]
                    && fns[3 * f + 2] == s->vf[3 * k + 2]) dup = 1;
            if (!dup) {
                memcpy(fns + 3 * nf, s->vf + 3 * k, 3 * sizeof(int));
                nf++;
            }
        }
    }
    return nf;
}

/* -------------------------------------------------------------- setup */

int or_setup(const or_problem *p, or_state **out) {
    if (p->fe_order < 1 || p->fe_order > 3) return -1;
    for (int d = 0; d < 3; ++d)
        if (p->mesh[d] < 2) return -2;
    or_state *s = calloc(1, sizeof *s);
    memcpy(s->lat, p->lat, sizeof s->lat);
    inv3(s->lat, s->inv, &s->detA);
    if (!(s->detA > 0)) { free(s); return -3; }
    memcpy(s->mesh, p->mesh, sizeof s->mesh);
    s->p = p->fe_order;
    s->nfs = (s->p == 1) ? 1 : (s->p == 2 ? 8 : 7);
    s->n_atoms = p->n_atoms;
    s->n_enr = p->n_enr;
    s->pos = malloc(sizeof(double) * 3 * (p->n_atoms + 1));
    memcpy(s->pos, p->pos, sizeof(double) * 3 * p->n_atoms);
    s->species = malloc(sizeof(int) * (p->n_atoms + 1));
    memcpy(s->species, p->species, sizeof(int) * p->n_atoms);
    int ne = p->n_enr + 1;
    s->enr_species = malloc(sizeof(int) * ne);
    s->enr_l = malloc(sizeof(int) * ne);
    s->enr_a = malloc(sizeof(double) * ne);
    s->enr_rc = malloc(sizeof(double) * ne);
    s->enr_re = malloc(sizeof(double) * ne);
    s->enr_nrad = calloc(ne, sizeof(int));
    s->enr_u = calloc(ne, sizeof(double *));
    s->enr_M = calloc(ne, sizeof(double *));
    const double *rad = p->enr_rad;
    for (int k = 0; k < p->n_enr; ++k) {
        s->enr_species[k] = p->enr_species[k];
        s->enr_l[k] = p->enr_l[k];
        s->enr_a[k] = p->enr_a[k];
        s->enr_rc[k] = p->enr_rc[k];
        s->enr_re[k] = p->enr_re[k];
        if (s->enr_l[k] < 0 || s->enr_l[k] > 3) { or_free(s); return -4; }
        int n = p->enr_nrad ? p->enr_nrad[k] : 0;
        if (n == 0) continue;
        if (n < 4 || !rad || !(s->enr_rc[k] > 0)) { or_free(s); return -5; }
        s->enr_nrad[k] = n;
        s->enr_u[k] = malloc(sizeof(double) * n);
        s->enr_M[k] = malloc(sizeof(double) * n);
        spline_fit(n, s->enr_rc[k], rad, s->enr_u[k], s->enr_M[k]);
        rad += n;
    }
    s->q_n = p->q_n;
    s->q_nref = p->q_nref;
    s->q_levels = p->q_levels;
    s->q_mode = p->q_mode;
    s->q_dist = p->q_dist;
    s->q_tol = p->q_tol;
    s->nel = (int64_t)s->mesh[0] * s->mesh[1] * s->mesh[2];
    s->nv = s->nel;

    /* enriched sets (section "Partition of unity enrichment functions") */
    int64_t cap = 64, nfn = 0;
    s->vf = malloc(sizeof(int) * 3 * cap);
    s->vf_off = malloc(sizeof(int64_t) * (s->nv + 1));
    for (int64_t v = 0; v < s->nv; ++v) {
        s->vf_off[v] = nfn;
        double xv[3];
        vertex_position(s, v, xv);
        for (int A = 0; A < s->n_atoms; ++A) {
            for (int k = 0; k < s->n_enr; ++k) {
                if (s->enr_species[k] != s->species[A]) continue;
                double dmin = min_image_distance(s, xv, s->pos + 3 * A, s->enr_re[k]);
                if (!(dmin < s->enr_re[k])) continue;
                for (int m = -s->enr_l[k]; m <= s->enr_l[k]; ++m) {
                    if (nfn == cap) {
                        cap *= 2;
                        s->vf = realloc(s->vf, sizeof(int) * 3 * cap);
                    }
                    s->vf[3 * nfn] = A;
                    s->vf[3 * nfn + 1] = k;
                    s->vf[3 * nfn + 2] = m;
                    nfn++;
                }
            }
        }
    }
    s->vf_off[s->nv] = nfn;
    s->dof_off = malloc(sizeof(int64_t) * (s->nv + 1));
    s->dof_off[0] = 0;
    for (int64_t v = 0; v < s->nv; ++v)
        s->dof_off[v + 1] = s->dof_off[v] + s->nfs + (s->vf_off[v + 1] - s->vf_off[v]);
    s->ndof = s->dof_off[s->nv];

    /* quadrature rule, element by element, leaves depth first */
    s->leaf_off = malloc(sizeof(int64_t) * (s->nel + 1));
    s->qp_off = malloc(sizeof(int64_t) * (s->nel + 1));
    leaf_list ll = {0};
    {
        int isortho = fabs(s->lat[1]) == 0 && fabs(s->lat[2]) == 0 && fabs(s->lat[3]) == 0
                      && fabs(s->lat[5]) == 0 && fabs(s->lat[6]) == 0 && fabs(s->lat[7]) == 0;
        if (s->q_mode == 0 && s->q_levels > 0 && !isortho) { or_free(s); return -5; }
        int *fns = malloc(sizeof(int) * 3 * (8 * (nfn + 1)));
        for (int64_t e = 0; e < s->nel; ++e) {
            s->leaf_off[e] = ll.n;
            int c0[3] = {0, 0, 0};
            if (s->q_mode == 0) {
                geom_cell(s, e, 0, c0, &ll);
            } else {
                int nf = element_functions(s, e, fns);
                error_cell(s, e, 0, c0, fns, nf, &ll);
            }
        }
        free(fns);
    }
    s->leaf_off[s->nel] = ll.n;
    s->nleaves = ll.n;
    s->leaf_level = ll.level;
    s->leaf_ijk = ll.ijk;
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int64_t e = 0; e <= s->nel; ++e) s->qp_off[e] = s->leaf_off[e] * nq3;
    s->nqp = s->qp_off[s->nel];
    s->gx = malloc(sizeof(double) * (s->q_n + 1));
    s->gw = malloc(sizeof(double) * (s->q_n + 1));
    if (s->q_n > 0) or_gauss_legendre(s->q_n, s->gx, s->gw);
    *out = s;
    return 0;
}

void or_free(or_state *s) {
    if (!s) return;
    free(s->pos); free(s->species);
    if (s->enr_u)
        for (int k = 0; k < s->n_enr; ++k) {
            free(s->enr_u[k]);
            free(s->enr_M[k]);
        }
    free(s->enr_u); free(s->enr_M); free(s->enr_nrad);
    free(s->enr_species); free(s->enr_l); free(s->enr_a); free(s->enr_rc); free(s->enr_re);
    free(s->vf_off); free(s->vf); free(s->dof_off);
    free(s->leaf_off); free(s->leaf_level); free(s->leaf_ijk); free(s->qp_off);
    free(s->gx); free(s->gw);
    free(s);
}

void or_sizes(const or_state *s, int64_t *o) {
    o[0] = s->nel;
    o[1] = s->nv;
    o[2] = s->ndof;
    o[3] = s->nqp;
    o[4] = s->nfs;
    o[5] = max_locals(s);
    o[6] = s->nleaves;
}

void or_dof_offset(const or_state *s, int64_t *out) {
    memcpy(out, s->dof_off, sizeof(int64_t) * (s->nv + 1));
}

int or_vertex_functions(const or_state *s, int64_t v, int *out) {
    int n = (int)(s->vf_off[v + 1] - s->vf_off[v]);
    memcpy(out, s->vf + 3 * s->vf_off[v], sizeof(int) * 3 * n);
    return n;
}

void or_set_positions(or_state *s, const double *pos) {
    memcpy(s->pos, pos, sizeof(double) * 3 * s->n_atoms);
}

/* qp j of leaf (lev, c): reference point and weight (Gauss points with the
 * first index fastest) */
static void leaf_point(const or_state *s, int lev, const int *c, int64_t j, double *xi, double *w) {
    int n = s->q_n;
    int k[3] = {(int)(j % n), (int)((j / n) % n), (int)(j / ((int64_t)n * n))};
    double h = 1.0 / (double)(1 << lev);
    double jac = s->detA / (8.0 * s->mesh[0] * s->mesh[1] * s->mesh[2]);
    double wt = h * h * h * jac;
    for (int d = 0; d < 3; ++d) {
        double lo, hi;
        cell_interval(lev, c[d], &lo, &hi);
        xi[d] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * s->gx[k[d]];
        wt *= s->gw[k[d]];
    }
    *w = wt;
}

void or_quadrature(const or_state *s, double *xyz, double *w, int64_t *elem_qp_off) {
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n, q = 0;
    for (int64_t e = 0; e < s->nel; ++e)
        for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
            for (int64_t j = 0; j < nq3; ++j, ++q) {
                double xi[3];
                leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w[q]);
                ref2phys(s, e, xi, xyz + 3 * q);
            }
    memcpy(elem_qp_off, s->qp_off, sizeof(int64_t) * (s->nel + 1));
}

void or_leaves(const or_state *s, int *level, int *ijk, int64_t *elem_leaf_off) {
    memcpy(level, s->leaf_level, sizeof(int) * s->nleaves);
    memcpy(ijk, s->leaf_ijk, sizeof(int) * 3 * s->nleaves);
    memcpy(elem_leaf_off, s->leaf_off, sizeof(int64_t) * (s->nel + 1));
}

int or_element_nloc(const or_state *s, int64_t e) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    free(L);
    return n;
}

void or_element_dofs(const or_state *s, int64_t e, int64_t *gdof, int *shift) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    for (int a = 0; a < n; ++a) {
        gdof[a] = L[a].g;
        for (int d = 0; d < 3; ++d) shift[3 * a + d] = L[a].shift[d];
    }
    free(L);
}

/* ------------------------------------------------------ element matrices */

/* H_e[a][b] = sum_q w_q (1/2 grad phi_a . grad phi_b + V_q phi_a phi_b),
 * S_e[a][b] = sum_q w_q phi_a phi_b  (eq. disceig3d restricted to one element;
 * real because the element-level functions are real). */
static void elem_mats(const or_state *s, int64_t e, const loc_fn *L, int n, const double *V,
                      double *He, double *Se) {
    double *val = malloc(sizeof(double) * n), *grad = malloc(sizeof(double) * 3 * n);
    memset(He, 0, sizeof(double) * n * n);
    memset(Se, 0, sizeof(double) * n * n);
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n, q = 0;
    for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
        for (int64_t j = 0; j < nq3; ++j, ++q) {
            double xi[3], w;
            leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
            basis_eval(s, e, L, n, xi, val, grad);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double gg = grad[3 * a] * grad[3 * b] + grad[3 * a + 1] * grad[3 * b + 1]
                              + grad[3 * a + 2] * grad[3 * b + 2];
                    He[a * n + b] += w * (0.5 * gg + V[q] * val[a] * val[b]);
                    Se[a * n + b] += w * val[a] * val[b];
                }
        }
    free(val);
    free(grad);
}

void or_element_matrices(const or_state *s, int64_t e, const double *V_elem, double *He, double *Se) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    elem_mats(s, e, L, n, V_elem, He, Se);
    free(L);
}

/* Bloch phase of a local function: exp(2 pi i kappa . n) */
static void phase(const double *kappa, const int *sh, double *re, double *im) {
    double t = 2.0 * OR_PI * (kappa[0] * sh[0] + kappa[1] * sh[1] + kappa[2] * sh[2]);
    *re = cos(t);
    *im = sin(t);
}

/* H[g_a][g_b] += conj(p_a) p_b H_e[a][b], the same for S (eq. disceig3d with
 * Bloch-periodic FE and PU functions). */
void or_assemble_dense(const or_state *s, const double *V, const double *kappa, double *H, double *S) {
    int64_t N = s->ndof;
    memset(H, 0, sizeof(double) * 2 * N * N);
    memset(S, 0, sizeof(double) * 2 * N * N);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *He = malloc(sizeof(double) * mx * mx), *Se = malloc(sizeof(double) * mx * mx);
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        elem_mats(s, e, L, n, V + s->qp_off[e], He, Se);
        for (int a = 0; a < n; ++a) {
            double par, pai;
            phase(kappa, L[a].shift, &par, &pai);
            for (int b = 0; b < n; ++b) {
                double pbr, pbi;
                phase(kappa, L[b].shift, &pbr, &pbi);
                double cr = par * pbr + pai * pbi, ci = par * pbi - pai * pbr; /* conj(pa) pb */
                int64_t idx = 2 * (L[a].g * N + L[b].g);
                H[idx] += cr * He[a * n + b];
                H[idx + 1] += ci * He[a * n + b];
                S[idx] += cr * Se[a * n + b];
                S[idx + 1] += ci * Se[a * n + b];
            }
        }
    }
    free(L); free(He); free(Se);
}

void or_assemble_block(const or_state *s, const double *V, const double *kappa, int64_t v,
                       int64_t w, double *Hb, double *Sb) {
    int64_t r0 = s->dof_off[v], nr = s->dof_off[v + 1] - r0;
    int64_t c0 = s->dof_off[w], nc = s->dof_off[w + 1] - c0;
    memset(Hb, 0, sizeof(double) * 2 * nr * nc);
    memset(Sb, 0, sizeof(double) * 2 * nr * nc);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *He = malloc(sizeof(double) * mx * mx), *Se = malloc(sizeof(double) * mx * mx);
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L), hasr = 0, hasc = 0;
        for (int a = 0; a < n; ++a) {
            if (L[a].g >= r0 && L[a].g < r0 + nr) hasr = 1;
            if (L[a].g >= c0 && L[a].g < c0 + nc) hasc = 1;
        }
        if (!hasr || !hasc) continue;
        elem_mats(s, e, L, n, V + s->qp_off[e], He, Se);
        for (int a = 0; a < n; ++a) {
            if (!(L[a].g >= r0 && L[a].g < r0 + nr)) continue;
            double par, pai;
            phase(kappa, L[a].shift, &par, &pai);
            for (int b = 0; b < n; ++b) {
                if (!(L[b].g >= c0 && L[b].g < c0 + nc)) continue;
                double pbr, pbi;
                phase(kappa, L[b].shift, &pbr, &pbi);
                double cr = par * pbr + pai * pbi, ci = par * pbi - pai * pbr;
                int64_t idx = 2 * ((L[a].g - r0) * nc + (L[b].g - c0));
                Hb[idx] += cr * He[a * n + b];
                Hb[idx + 1] += ci * He[a * n + b];
                Sb[idx] += cr * Se[a * n + b];
                Sb[idx + 1] += ci * Se[a * n + b];
            }
        }
    }
    free(L); free(He); free(Se);
}

/* ----------------------------------------- Bloch-periodic enrichment basis */

/* Values and gradients, real parts vr, gr and imaginary parts vi, gi, of the
 * element's basis when the enrichment is Bloch-periodic (eq. Psi with
 * f(R) = exp(i k.R)): the classical FE functions as in basis_eval (real),
 * and PU functions times Psi^k (or_enrichment_bloch).  The PU functions carry
 * no boundary phase in this form: they are periodic, so that their product
 * with the Bloch-periodic Psi^k is Bloch-periodic. */
static void basis_eval_bloch(const or_state *s, int64_t e, const loc_fn *L, int nloc, const double *xi,
                             const double *kappa, double *vr, double *vi, double *gr, double *gi) {
    double x[3];
    ref2phys(s, e, xi, x);
    basis_eval(s, e, L, nloc, xi, vr, gr);   /* FE rows; enriched rows replaced below */
    for (int a = 0; a < nloc; ++a) {
        vi[a] = 0.0;
        for (int c = 0; c < 3; ++c) gi[3 * a + c] = 0.0;
        if (L[a].kind == 0) continue;
        double M = 1.0, dxi[3] = {1.0, 1.0, 1.0};
        for (int d = 0; d < 3; ++d) {
            double lv, ld;
            or_lagrange(1, (L[a].corner >> d) & 1, xi[d], &lv, &ld);
            for (int k = 0; k < 3; ++k) dxi[k] *= (k == d) ? ld : lv;
            M *= lv;
        }
        double gM[3], psi[2], gpsi[6];
        ref_grad(s, dxi, gM);
        or_enrichment_bloch(s, L[a].atom, L[a].desc, L[a].m, x, kappa, psi, gpsi);
        vr[a] = M * psi[0];
        vi[a] = M * psi[1];
        for (int c = 0; c < 3; ++c) {
            gr[3 * a + c] = gM[c] * psi[0] + M * gpsi[c];
            gi[3 * a + c] = gM[c] * psi[1] + M * gpsi[3 + c];
        }
    }
}

/* Complex element matrices of the Bloch-enriched basis (eq. disceig3d on one
 * element), interleaved (Re, Im), n x n:
 *   H_e[a][b] = sum_q w_q (1/2 conj(grad phi_a) . grad phi_b + V_q conj(phi_a) phi_b),
 *   S_e[a][b] = sum_q w_q conj(phi_a) phi_b. */
static void elem_mats_bloch(const or_state *s, int64_t e, const loc_fn *L, int n, const double *V,
                            const double *kappa, double *He, double *Se) {
    double *vr = malloc(sizeof(double) * n), *vi = malloc(sizeof(double) * n);
    double *gr = malloc(sizeof(double) * 3 * n), *gi = malloc(sizeof(double) * 3 * n);
    memset(He, 0, sizeof(double) * 2 * n * n);
    memset(Se, 0, sizeof(double) * 2 * n * n);
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n, q = 0;
    for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
        for (int64_t j = 0; j < nq3; ++j, ++q) {
            double xi[3], w;
            leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
            basis_eval_bloch(s, e, L, n, xi, kappa, vr, vi, gr, gi);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    /* conj(u) v = (ur ur' + ui vi') + i (ur vi' - ui vr') */
                    double pr = vr[a] * vr[b] + vi[a] * vi[b], pi = vr[a] * vi[b] - vi[a] * vr[b];
                    double ggr = 0.0, ggi = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        ggr += gr[3 * a + c] * gr[3 * b + c] + gi[3 * a + c] * gi[3 * b + c];
                        ggi += gr[3 * a + c] * gi[3 * b + c] - gi[3 * a + c] * gr[3 * b + c];
                    }
                    He[2 * (a * n + b)] += w * (0.5 * ggr + V[q] * pr);
                    He[2 * (a * n + b) + 1] += w * (0.5 * ggi + V[q] * pi);
                    Se[2 * (a * n + b)] += w * pr;
                    Se[2 * (a * n + b) + 1] += w * pi;
                }
        }
    free(vr); free(vi); free(gr); free(gi);
}

void or_element_matrices_bloch(const or_state *s, int64_t e, const double *V_elem, const double *kappa,
                               double *He, double *Se) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    elem_mats_bloch(s, e, L, n, V_elem, kappa, He, Se);
    free(L);
}

/* Global matrices of the Bloch-enriched basis restricted to rows [r0, r0+nr)
 * and columns [c0, c0+nc): H[g_a][g_b] += conj(p_a) p_b H_e[a][b] with the
 * boundary phase p_a = exp(2 pi i kappa.n_a) of the classical FE functions
 * and p_a = 1 for the enriched ones (periodic PU), the same for S. */
static void assemble_bloch(const or_state *s, const double *V, const double *kappa, int64_t r0, int64_t nr,
                           int64_t c0, int64_t nc, double *H, double *S) {
    memset(H, 0, sizeof(double) * 2 * nr * nc);
    memset(S, 0, sizeof(double) * 2 * nr * nc);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *He = malloc(sizeof(double) * 2 * mx * mx), *Se = malloc(sizeof(double) * 2 * mx * mx);
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L), hasr = 0, hasc = 0;
        for (int a = 0; a < n; ++a) {
            if (L[a].g >= r0 && L[a].g < r0 + nr) hasr = 1;
            if (L[a].g >= c0 && L[a].g < c0 + nc) hasc = 1;
        }
        if (!hasr || !hasc) continue;
        elem_mats_bloch(s, e, L, n, V + s->qp_off[e], kappa, He, Se);
        for (int a = 0; a < n; ++a) {
            if (!(L[a].g >= r0 && L[a].g < r0 + nr)) continue;
            double par = 1.0, pai = 0.0;
            if (L[a].kind == 0) phase(kappa, L[a].shift, &par, &pai);
            for (int b = 0; b < n; ++b) {
                if (!(L[b].g >= c0 && L[b].g < c0 + nc)) continue;
                double pbr = 1.0, pbi = 0.0;
                if (L[b].kind == 0) phase(kappa, L[b].shift, &pbr, &pbi);
                double cr = par * pbr + pai * pbi, ci = par * pbi - pai * pbr; /* conj(pa) pb */
                const double *h = He + 2 * (a * n + b), *sv = Se + 2 * (a * n + b);
                int64_t idx = 2 * ((L[a].g - r0) * nc + (L[b].g - c0));
                H[idx] += cr * h[0] - ci * h[1];
                H[idx + 1] += cr * h[1] + ci * h[0];
                S[idx] += cr * sv[0] - ci * sv[1];
                S[idx + 1] += cr * sv[1] + ci * sv[0];
            }
        }
    }
    free(L); free(He); free(Se);
}

void or_assemble_dense_bloch(const or_state *s, const double *V, const double *kappa, double *H, double *S) {
    assemble_bloch(s, V, kappa, 0, s->ndof, 0, s->ndof, H, S);
}

void or_assemble_block_bloch(const or_state *s, const double *V, const double *kappa, int64_t v, int64_t w,
                             double *Hb, double *Sb) {
    int64_t r0 = s->dof_off[v], nr = s->dof_off[v + 1] - r0;
    int64_t c0 = s->dof_off[w], nc = s->dof_off[w + 1] - c0;
    assemble_bloch(s, V, kappa, r0, nr, c0, nc, Hb, Sb);
}

/* ---------------------------------------------------------------- adjoint */

/* L = Re sum_ij conj(P_ij) H_ij + Re sum_ij conj(Q_ij) S_ij.  With
 * Pt_e[a][b] = Re(p_a P[g_a][g_b] conj(p_b)) (and Qt likewise),
 * L = sum_e sum_ab Pt_e[a][b] H_e[a][b] + Qt_e[a][b] S_e[a][b], so
 *   dL/dV_q = w_q sum_ab Pt[a][b] phi_a phi_b            (the density n(x_q) w_q,
 *             cf. eq. rhoe when P is the occupied-state density matrix), and
 *   dL/dtau_A = sum_q w_q sum_ab Pt[a][b] (1/2 (grad phi'_a . grad phi_b + grad phi_a . grad phi'_b)
 *               + V_q (phi'_a phi_b + phi_a phi'_b)) + Qt[a][b] (phi'_a phi_b + phi_a phi'_b),
 * where phi' is the derivative of the function with respect to the centre of
 * its enrichment: d(M_c Psi)/dtau = -M_c grad Psi and
 * d(grad(M_c Psi))/dtau_k = -(grad M_c d_k Psi + M_c grad d_k Psi).
 * The quadrature rule, the enriched sets and V are held fixed. */
/* The adjoint contribution of one element: Ploc and Qloc hold the entries
 * P[g_a][g_b] (complex, n x n) of the element's local functions; Qloc may be
 * NULL.  Adds w_q phi^T Pt phi to dLdV_elem[q] (element-local points) and the
 * element's share of dL/dtau to dLdR. */
static void backward_element(const or_state *s, int64_t e, const loc_fn *L, int n, const double *V,
                             const double *kappa, const double *Ploc, const double *Qloc,
                             double *dLdV, double *dLdR) {
    double *Pt = malloc(sizeof(double) * n * n), *Qt = malloc(sizeof(double) * n * n);
    double *val = malloc(sizeof(double) * n), *grad = malloc(sizeof(double) * 3 * n);
    double *dval = malloc(sizeof(double) * 3 * n);   /* d phi_a / d tau_k */
    double *dgrad = malloc(sizeof(double) * 9 * n);  /* d (d_j phi_a) / d tau_k at [9a + 3k + j] */
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int a = 0; a < n; ++a) {
        double par, pai;
        phase(kappa, L[a].shift, &par, &pai);
        for (int b = 0; b < n; ++b) {
            double pbr, pbi;
            phase(kappa, L[b].shift, &pbr, &pbi);
            /* Re(p_a X conj(p_b)) = Re(X) Re(p_a conj p_b) - Im(X) Im(p_a conj p_b) */
            double zr = par * pbr + pai * pbi, zi = pai * pbr - par * pbi;
            int64_t idx = 2 * ((int64_t)a * n + b);
            Pt[a * n + b] = Ploc[idx] * zr - Ploc[idx + 1] * zi;
            Qt[a * n + b] = Qloc ? (Qloc[idx] * zr - Qloc[idx + 1] * zi) : 0.0;
        }
    }
    int64_t q = 0;
    for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
        for (int64_t j = 0; j < nq3; ++j, ++q) {
            double xi[3], w, x[3];
            leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
            basis_eval(s, e, L, n, xi, val, grad);
            ref2phys(s, e, xi, x);
            for (int a = 0; a < n; ++a) {
                memset(dval + 3 * a, 0, sizeof(double) * 3);
                memset(dgrad + 9 * a, 0, sizeof(double) * 9);
                if (L[a].kind != 1) continue;
                double M = 1.0, dxi[3] = {1.0, 1.0, 1.0}, gM[3], psi, gpsi[3], hpsi[9];
                for (int d = 0; d < 3; ++d) {
                    double lv, ld;
                    or_lagrange(1, (L[a].corner >> d) & 1, xi[d], &lv, &ld);
                    for (int k = 0; k < 3; ++k) dxi[k] *= (k == d) ? ld : lv;
                    M *= lv;
                }
                ref_grad(s, dxi, gM);
                or_enrichment(s, L[a].atom, L[a].desc, L[a].m, x, &psi, gpsi, hpsi);
                for (int k = 0; k < 3; ++k) {
                    dval[3 * a + k] = -M * gpsi[k];
                    for (int jj = 0; jj < 3; ++jj)
                        dgrad[9 * a + 3 * k + jj] = -(gM[jj] * gpsi[k] + M * hpsi[jj * 3 + k]);
                }
            }
            double dv = 0.0;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) dv += Pt[a * n + b] * val[a] * val[b];
            dLdV[q] += w * dv;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    for (int side = 0; side < 2; ++side) {
                        /* side 0 differentiates phi_a, side 1 differentiates phi_b */
                        int d = side == 0 ? a : b, o = side == 0 ? b : a;
                        if (L[d].kind != 1) continue;
                        int A = L[d].atom;
                        for (int k = 0; k < 3; ++k) {
                            double gg = 0.0;
                            for (int jj = 0; jj < 3; ++jj)
                                gg += dgrad[9 * d + 3 * k + jj] * grad[3 * o + jj];
                            double pv = dval[3 * d + k] * val[o];
                            dLdR[3 * A + k] += w * (Pt[a * n + b] * (0.5 * gg + V[q] * pv)
                                                    + Qt[a * n + b] * pv);
                        }
                    }
                }
        }
    free(Pt); free(Qt); free(val); free(grad); free(dval); free(dgrad);
}

void or_backward_dense(const or_state *s, const double *V, const double *kappa, const double *P,
                       const double *Q, double *dLdV, double *dLdR) {
    int64_t N = s->ndof;
    memset(dLdV, 0, sizeof(double) * s->nqp);
    memset(dLdR, 0, sizeof(double) * 3 * s->n_atoms);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *Pl = malloc(sizeof(double) * 2 * mx * mx), *Ql = malloc(sizeof(double) * 2 * mx * mx);
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                for (int t = 0; t < 2; ++t) {
                    Pl[2 * (a * n + b) + t] = P[2 * (L[a].g * N + L[b].g) + t];
                    Ql[2 * (a * n + b) + t] = Q ? Q[2 * (L[a].g * N + L[b].g) + t] : 0.0;
                }
        backward_element(s, e, L, n, V + s->qp_off[e], kappa, Pl, Q ? Ql : NULL,
                         dLdV + s->qp_off[e], dLdR);
    }
    free(L); free(Pl); free(Ql);
}

void or_backward_element(const or_state *s, int64_t e, const double *V_elem, const double *kappa,
                         const double *Ploc, const double *Qloc, double *dLdV_elem, double *dLdR) {
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    int n = element_locals(s, e, L);
    memset(dLdV_elem, 0, sizeof(double) * (s->qp_off[e + 1] - s->qp_off[e]));
    memset(dLdR, 0, sizeof(double) * 3 * s->n_atoms);
    backward_element(s, e, L, n, V_elem, kappa, Ploc, Qloc, dLdV_elem, dLdR);
    free(L);
}

/* ----------------------------------------------------------- sparsity */

/* number of (i, j) DOF pairs that share an element: the nonzero pattern of S
 * (section "Self-consistent calculations", sparsity table) */
int64_t or_pattern_nnz(const or_state *s) {
    int64_t N = s->ndof, nnz = 0;
    unsigned char *mark = calloc((size_t)(N * N), 1);
    loc_fn *L = malloc(sizeof(loc_fn) * max_locals(s));
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) mark[L[a].g * N + L[b].g] = 1;
    }
    for (int64_t k = 0; k < N * N; ++k) nnz += mark[k];
    free(mark);
    free(L);
    return nnz;
}

/* ------------------------------------------- separable nonlocal potential */

/* Projector function of descriptor d (2l+1 of them, m = -l..l) centred at
 * the origin: v(r) = exp(-a |r|^2) (1 - |r|^2/rc^2)^3 S_lm(r) for |r| < rc,
 * 0 beyond (the radial form of the enrichment descriptors; synthetic stand-ins
 * for the projectors of a separable pseudopotential). */
static double projector_value(int l, int m, double a, double rc, const double *r) {
    double sq = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    if (sq >= rc * rc) return 0.0;
    double c = 1.0 - sq / (rc * rc), S;
    or_solid_harmonic(l, m, r, &S, NULL, NULL);
    return exp(-a * sq) * c * c * c * S;
}

/* Coefficients of the separable nonlocal term (eq. disceig3d):
 *   f_J^i = int_cell phi_i^*(x) sum_n exp(i k . a_n) v_J(x - tau_A - a_n) dx
 * for every projector function J = (atom A of the descriptor's species,
 * descriptor, m), in descriptor order, atoms in order, m = -l..l; with
 * k . a_n = 2 pi kappa . n.  phi_i^* on element e is conj(p_a) N_a (the Bloch
 * phase of local function a), so
 *   f_J^i = sum_e sum_{a -> i} conj(p_a) sum_q w_q N_a(x_q) P_J(x_q),
 *   P_J(x) = sum_n exp(2 pi i kappa . n) v_J(x - tau_A - a_n).
 * F: n_fun x N complex (re, im), row J.  Returns n_fun. */
/* f_J^i over the basis of the periodic (bloch = 0) or the Bloch-periodic
 * (bloch = 1) enrichment: the conjugate of p_a phi_a, with the boundary phase
 * p_a on the classical FE functions (and, in the periodic form, on the PU
 * functions too), times the Bloch sum of the projector function. */
static int nonlocal_f(const or_state *s, const double *kappa, int n_proj, const int *proj_species, const int *proj_l,
                      const double *proj_a, const double *proj_rc, double *F, int bloch) {
    /* projector functions */
    int nfun = 0;
    for (int d = 0; d < n_proj; ++d)
        for (int A = 0; A < s->n_atoms; ++A)
            if (s->species[A] == proj_species[d]) nfun += 2 * proj_l[d] + 1;
    if (!F) return nfun;
    int *fa = malloc(sizeof(int) * (nfun + 1)), *fd = malloc(sizeof(int) * (nfun + 1)),
        *fm = malloc(sizeof(int) * (nfun + 1));
    int J = 0;
    for (int d = 0; d < n_proj; ++d)
        for (int A = 0; A < s->n_atoms; ++A)
            if (s->species[A] == proj_species[d])
                for (int m = -proj_l[d]; m <= proj_l[d]; ++m) {
                    fa[J] = A;
                    fd[J] = d;
                    fm[J] = m;
                    ++J;
                }
    int64_t N = s->ndof;
    memset(F, 0, sizeof(double) * 2 * (size_t)nfun * N);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *val = malloc(sizeof(double) * mx), *grad = malloc(sizeof(double) * 3 * mx);
    double *vim = calloc(mx, sizeof(double)), *gim = malloc(sizeof(double) * 3 * mx);
    double *Pre = malloc(sizeof(double) * (nfun + 1)), *Pim = malloc(sizeof(double) * (nfun + 1));
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
            for (int64_t j = 0; j < nq3; ++j) {
                double xi[3], w, x[3];
                leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
                ref2phys(s, e, xi, x);
                if (bloch)
                    basis_eval_bloch(s, e, L, n, xi, kappa, val, vim, grad, gim);
                else
                    basis_eval(s, e, L, n, xi, val, grad);
                /* Bloch sums of the projector functions at x */
                double ux[3];
                cart2red(s, x, ux);
                for (int J2 = 0; J2 < nfun; ++J2) {
                    const int d = fd[J2];
                    const double *tau = s->pos + 3 * fa[J2];
                    int lo[3], hi[3];
                    image_range(s, tau, ux, ux, proj_rc[d], lo, hi);
                    double re = 0.0, im = 0.0;
                    for (int n3 = lo[2]; n3 <= hi[2]; ++n3)
                        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
                            for (int n1 = lo[0]; n1 <= hi[0]; ++n1) {
                                double nn[3] = {(double)n1, (double)n2, (double)n3}, R[3], r[3];
                                red2cart(s, nn, R);
                                for (int c = 0; c < 3; ++c) r[c] = x[c] - tau[c] - R[c];
                                double v = projector_value(proj_l[d], fm[J2], proj_a[d], proj_rc[d], r);
                                if (v == 0.0) continue;
                                double t = 2.0 * OR_PI * (kappa[0] * n1 + kappa[1] * n2 + kappa[2] * n3);
                                re += cos(t) * v;
                                im += sin(t) * v;
                            }
                    Pre[J2] = re;
                    Pim[J2] = im;
                }
                for (int a = 0; a < n; ++a) {
                    double par = 1.0, pai = 0.0;
                    if (!bloch || L[a].kind == 0) phase(kappa, L[a].shift, &par, &pai);
                    /* w conj(p_a phi_a) P_J */
                    double qr = par * val[a] - pai * vim[a], qi = par * vim[a] + pai * val[a];
                    double cr = w * qr, ci = -w * qi;
                    for (int J2 = 0; J2 < nfun; ++J2) {
                        double *f = F + 2 * ((size_t)J2 * N + L[a].g);
                        f[0] += cr * Pre[J2] - ci * Pim[J2];
                        f[1] += cr * Pim[J2] + ci * Pre[J2];
                    }
                }
            }
    }
    free(L); free(val); free(grad); free(vim); free(gim); free(Pre); free(Pim); free(fa); free(fd); free(fm);
    return nfun;
}

int or_nonlocal_f(const or_state *s, const double *kappa, int n_proj, const int *proj_species, const int *proj_l,
                  const double *proj_a, const double *proj_rc, double *F) {
    return nonlocal_f(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, F, 0);
}

int or_nonlocal_f_bloch(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                        const int *proj_l, const double *proj_a, const double *proj_rc, double *F) {
    return nonlocal_f(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, F, 1);
}

/* The separable nonlocal term of eq. disceig3d as a dense matrix:
 *   Vnl_ij = sum_J h_J f_J^i conj(f_J^j),
 * with h_J the weight of J's descriptor.  Vnl: N x N complex (re, im). */
static void nonlocal_dense(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                           const int *proj_l, const double *proj_a, const double *proj_rc, const double *proj_h,
                           double *Vnl, int bloch) {
    int nfun = nonlocal_f(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, NULL, bloch);
    int64_t N = s->ndof;
    double *F = malloc(sizeof(double) * 2 * ((size_t)nfun * N + 1));
    nonlocal_f(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, F, bloch);
    double *h = malloc(sizeof(double) * (nfun + 1));
    int J = 0;
    for (int d = 0; d < n_proj; ++d)
        for (int A = 0; A < s->n_atoms; ++A)
            if (s->species[A] == proj_species[d])
                for (int m = -proj_l[d]; m <= proj_l[d]; ++m) h[J++] = proj_h[d];
    memset(Vnl, 0, sizeof(double) * 2 * (size_t)N * N);
    for (int J2 = 0; J2 < nfun; ++J2) {
        const double *f = F + 2 * (size_t)J2 * N;
        for (int64_t i = 0; i < N; ++i) {
            if (f[2 * i] == 0.0 && f[2 * i + 1] == 0.0) continue;
            for (int64_t j = 0; j < N; ++j) {
                /* h f_i conj(f_j) */
                double ar = f[2 * i], ai = f[2 * i + 1], br = f[2 * j], bi = f[2 * j + 1];
                Vnl[2 * (i * N + j)] += h[J2] * (ar * br + ai * bi);
                Vnl[2 * (i * N + j) + 1] += h[J2] * (ai * br - ar * bi);
            }
        }
    }
    free(F);
    free(h);
}

void or_nonlocal_dense(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                       const int *proj_l, const double *proj_a, const double *proj_rc, const double *proj_h,
                       double *Vnl) {
    nonlocal_dense(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, proj_h, Vnl, 0);
}

void or_nonlocal_dense_bloch(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                             const int *proj_l, const double *proj_a, const double *proj_rc, const double *proj_h,
                             double *Vnl) {
    nonlocal_dense(s, kappa, n_proj, proj_species, proj_l, proj_a, proj_rc, proj_h, Vnl, 1);
}


/* ------------------------------------------- self-consistent field pieces */

/* Section "Self-consistent calculations" and eqs. poisson, veff: the
 * Coulomb potential is the solution of a Poisson problem, here posed on the
 * classical FE functions (periodic, Gamma: no boundary phase); its vectors are
 * indexed v * nfs + slot. */
int64_t or_n_fe_dof(const or_state *s) { return s->nv * s->nfs; }

/* b_i = sum_q w_q phi_i(x_q) f(x_q) over the classical FE functions, f given at
 * the rule's points in canonical order. */
void or_fe_load(const or_state *s, const double *f, double *b) {
    memset(b, 0, sizeof(double) * s->nv * s->nfs);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        int64_t q = s->qp_off[e];
        for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
            for (int64_t j = 0; j < nq3; ++j, ++q) {
                double xi[3], w;
                leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
                for (int a = 0; a < n; ++a) {
                    if (L[a].kind != 0) continue;
                    double v, g[3];
                    fe_function(s, &L[a], xi, &v, g);
                    b[L[a].fe] += w * v * f[q];
                }
            }
    }
    free(L);
}

/* u_h(x_q) = sum_i u_i phi_i(x_q) at every point of the rule. */
void or_fe_eval(const or_state *s, const double *u, double *out) {
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        int64_t q = s->qp_off[e];
        for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
            for (int64_t j = 0; j < nq3; ++j, ++q) {
                double xi[3], w, acc = 0.0;
                leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
                for (int a = 0; a < n; ++a) {
                    if (L[a].kind != 0) continue;
                    double v, g[3];
                    fe_function(s, &L[a], xi, &v, g);
                    acc += u[L[a].fe] * v;
                }
                out[q] = acc;
            }
    }
    free(L);
}

/* K_ij = sum_q w_q grad phi_i . grad phi_j over the classical FE functions
 * (dense, row-major, n_fe_dof x n_fe_dof). */
void or_fe_stiffness(const or_state *s, double *K) {
    int64_t N = s->nv * s->nfs;
    memset(K, 0, sizeof(double) * N * N);
    int mx = max_locals(s);
    loc_fn *L = malloc(sizeof(loc_fn) * mx);
    double *val = malloc(sizeof(double) * mx), *grad = malloc(sizeof(double) * 3 * mx);
    int64_t nq3 = (int64_t)s->q_n * s->q_n * s->q_n;
    for (int64_t e = 0; e < s->nel; ++e) {
        int n = element_locals(s, e, L);
        for (int64_t lf = s->leaf_off[e]; lf < s->leaf_off[e + 1]; ++lf)
            for (int64_t j = 0; j < nq3; ++j) {
                double xi[3], w;
                leaf_point(s, s->leaf_level[lf], s->leaf_ijk + 3 * lf, j, xi, &w);
                for (int a = 0; a < n; ++a)
                    if (L[a].kind == 0) fe_function(s, &L[a], xi, &val[a], grad + 3 * a);
                for (int a = 0; a < n; ++a) {
                    if (L[a].kind != 0) continue;
                    for (int b = 0; b < n; ++b) {
                        if (L[b].kind != 0) continue;
                        K[L[a].fe * N + L[b].fe] += w * (grad[3 * a] * grad[3 * b] + grad[3 * a + 1] * grad[3 * b + 1]
                                                         + grad[3 * a + 2] * grad[3 * b + 2]);
                    }
                }
            }
    }
    free(L); free(val); free(grad);
}

/* Local-density exchange-correlation of the unpolarised electron gas (the
 * LDA the paper names in section "Kohn-Sham density functional theory"): at
 * electron density n (bohr^-3), r_s = (3 / (4 pi n))^(1/3),
 *   exchange (Slater):  e_x = -(3/4) (3 n / pi)^(1/3),  v_x = (4/3) e_x;
 *   correlation: the Perdew-Zunger (1981) fit of the Ceperley-Alder data,
 *     r_s >= 1:  e_c = g / (1 + b1 sqrt(r_s) + b2 r_s),
 *                v_c = e_c (1 + 7/6 b1 sqrt(r_s) + 4/3 b2 r_s) / (1 + b1 sqrt(r_s) + b2 r_s),
 *     r_s <  1:  e_c = A ln r_s + B + C r_s ln r_s + D r_s,
 *                v_c = A ln r_s + (B - A/3) + 2/3 C r_s ln r_s + (2 D - C)/3 r_s,
 *   g = -0.1423, b1 = 1.0529, b2 = 0.3334, A = 0.0311, B = -0.048, C = 0.0020,
 *   D = -0.0116 (hartree).  exc is the energy per electron, vxc = d(n exc)/dn;
 * n <= 1e-30 gives zero. */
void or_lda(int64_t n, const double *rho, double *vxc, double *exc) {
    for (int64_t i = 0; i < n; ++i) {
        double d = rho[i];
        if (!(d > 1e-30)) {
            vxc[i] = 0.0;
            if (exc) exc[i] = 0.0;
            continue;
        }
        double rs = cbrt(3.0 / (4.0 * OR_PI * d));
        double ex = -0.75 * cbrt(3.0 * d / OR_PI), vx = 4.0 / 3.0 * ex;
        double ec, vc;
        if (rs >= 1.0) {
            const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
            double sr = sqrt(rs), den = 1.0 + b1 * sr + b2 * rs;
            ec = g / den;
            vc = ec * (1.0 + 7.0 / 6.0 * b1 * sr + 4.0 / 3.0 * b2 * rs) / den;
        } else {
            const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
            double lr = log(rs);
            ec = A * lr + B + C * rs * lr + D * rs;
            vc = A * lr + (B - A / 3.0) + 2.0 / 3.0 * C * rs * lr + (2.0 * D - C) / 3.0 * rs;
        }
        vxc[i] = vx + vc;
        if (exc) exc[i] = ex + ec;
    }
}
