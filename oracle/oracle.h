/*
 * PUFE assembly oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of what the PUFE
 * hot path computes (Pask & Sukumar, "Partition of unity finite element
 * method for quantum mechanical materials calculations"):
 *   - the enriched basis of the PUFE trial function (eq. psih / pufebasis),
 *   - the adaptive per-element quadrature rule (section "Adaptive quadrature"),
 *   - the Galerkin matrices H and S of the discrete generalized eigenproblem
 *     (eq. disceig3d) under Bloch boundary conditions (eq. bloch, wbpspace),
 *   - the adjoint of that assembly (dL/dV and dL/dtau for L = Re<P,H> + Re<Q,S>),
 *   - the separable nonlocal term of H (eq. disceig3d),
 *   - tabulated radial functions: a cubic spline through samples of the
 *     radial times the C^3 cutoff (section "Partition of unity enrichment
 *     functions").
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the HIP library.
 */
#ifndef PUFE_ORACLE_H
#define PUFE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double lat[9];        /* rows a_1, a_2, a_3 (bohr) */
    int mesh[3];          /* elements along each lattice vector */
    int fe_order;         /* 1 trilinear, 2 triquadratic, 3 32-node cubic serendipity */
    int n_atoms;
    const double *pos;    /* n_atoms x 3 Cartesian */
    const int *species;   /* n_atoms */
    int n_enr;            /* enrichment descriptors */
    const int *enr_species, *enr_l;
    const double *enr_a, *enr_rc, *enr_re;
    int q_n, q_nref, q_levels, q_mode;  /* q_mode 0 = geometric, 1 = error-driven */
    double q_dist, q_tol;
    /* tabulated radials (may be NULL: every descriptor analytic): enr_nrad[k]
     * samples of descriptor k (0 = analytic radial), concatenated in enr_rad */
    const int *enr_nrad;
    const double *enr_rad;
} or_problem;

typedef struct or_state or_state;

/* Returns 0 on success, a negative code on invalid input. */
int or_setup(const or_problem *p, or_state **out);
void or_free(or_state *s);
/* sizes: [n_elem, n_vertex, n_dof, n_qp, n_fe_slots, max_nloc, n_leaves] */
void or_sizes(const or_state *s, int64_t *out7);
void or_dof_offset(const or_state *s, int64_t *out /* n_vertex+1 */);
/* enriched functions of vertex v: (atom, desc, m) triples, returns count */
int or_vertex_functions(const or_state *s, int64_t v, int *out /* 3*count */);
void or_quadrature(const or_state *s, double *xyz, double *w, int64_t *elem_qp_off);
/* leaves: level and integer coordinates at that level, element-major DFS */
void or_leaves(const or_state *s, int *level, int *ijk, int64_t *elem_leaf_off);
int or_element_nloc(const or_state *s, int64_t e);
/* global dof and lattice shift (3 ints) of each local function of element e */
void or_element_dofs(const or_state *s, int64_t e, int64_t *gdof, int *shift);
/* real element matrices (nloc x nloc, row-major) from V at the element's qps */
void or_element_matrices(const or_state *s, int64_t e, const double *V_elem,
                         double *He, double *Se);
/* dense complex Bloch-periodic H, S (N x N interleaved re,im), kappa reduced */
void or_assemble_dense(const or_state *s, const double *V, const double *kappa,
                       double *H, double *S);
/* one (row vertex, col vertex) block of H and S, b_v x b_w complex */
void or_assemble_block(const or_state *s, const double *V, const double *kappa,
                       int64_t v, int64_t w, double *Hb, double *Sb);
/* adjoint of the assembly; P, Q dense N x N complex (Q may be NULL) */
void or_backward_dense(const or_state *s, const double *V, const double *kappa,
                       const double *P, const double *Q, double *dLdV, double *dLdR);
/* adjoint contribution of element e: Ploc/Qloc are the entries P[g_a][g_b]
 * (n x n complex) of its local functions, Qloc may be NULL; dLdV_elem gets the
 * element's points, dLdR (n_atoms x 3) its share of the force */
void or_backward_element(const or_state *s, int64_t e, const double *V_elem, const double *kappa,
                         const double *Ploc, const double *Qloc, double *dLdV_elem, double *dLdR);
/* move the enrichment centres only (rule and enriched sets stay frozen) */
void or_set_positions(or_state *s, const double *pos);
/* basis of element e at reference point xi: values and Cartesian gradients */
void or_basis_at(const or_state *s, int64_t e, const double *xi, double *val, double *grad);
/* enrichment function value, gradient, Hessian at x */
void or_enrichment(const or_state *s, int atom, int desc, int m, const double *x,
                   double *val, double *grad, double *hess);
/* Bloch-periodic enrichment (eq. Psi with f(R) = exp(i k.R)), periodic PU:
 * Psi^k at x (val[2] = Re, Im; grad[6] = Re parts, then Im parts); complex
 * element matrices (n x n interleaved); dense N x N and one vertex block of
 * the global H, S, with the boundary phase on the classical FE functions only */
void or_enrichment_bloch(const or_state *s, int atom, int desc, int m, const double *x, const double *kappa,
                         double *val, double *grad);
void or_element_matrices_bloch(const or_state *s, int64_t e, const double *V_elem, const double *kappa,
                               double *He, double *Se);
void or_assemble_dense_bloch(const or_state *s, const double *V, const double *kappa, double *H, double *S);
void or_assemble_block_bloch(const or_state *s, const double *V, const double *kappa, int64_t v, int64_t w,
                             double *Hb, double *Sb);
/* self-consistent field pieces (section "Self-consistent calculations",
 * eqs. poisson, veff): classical FE space vectors indexed v * nfs + slot,
 * periodic (Gamma); load vector b_i = sum_q w_q phi_i f_q, evaluation
 * u_h(x_q), dense stiffness matrix, and the LDA exchange-correlation */
int64_t or_n_fe_dof(const or_state *s);
void or_fe_load(const or_state *s, const double *f, double *b);
void or_fe_eval(const or_state *s, const double *u, double *out);
void or_fe_stiffness(const or_state *s, double *K);
void or_lda(int64_t n, const double *rho, double *vxc, double *exc);
/* building blocks exposed for the pins */
void or_gauss_legendre(int n, double *x, double *w);
void or_lagrange(int p, int j, double t, double *val, double *der);
void or_solid_harmonic(int l, int m, const double *r, double *val, double *grad, double *hess);
/* separable nonlocal term (eq. disceig3d): projector descriptors (species,
 * l, a, rc[, h]) as parallel arrays; or_nonlocal_f gives the coefficients
 * f_J^i (n_fun x N complex; F = NULL returns n_fun only), or_nonlocal_dense
 * the N x N complex matrix sum_J h_J f_J^i conj(f_J^j) */
int or_nonlocal_f(const or_state *s, const double *kappa, int n_proj, const int *proj_species, const int *proj_l,
                  const double *proj_a, const double *proj_rc, double *F);
void or_nonlocal_dense(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                       const int *proj_l, const double *proj_a, const double *proj_rc, const double *proj_h,
                       double *Vnl);
/* the same over the basis of the Bloch-periodic enrichment */
int or_nonlocal_f_bloch(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                        const int *proj_l, const double *proj_a, const double *proj_rc, double *F);
void or_nonlocal_dense_bloch(const or_state *s, const double *kappa, int n_proj, const int *proj_species,
                             const int *proj_l, const double *proj_a, const double *proj_rc, const double *proj_h,
                             double *Vnl);
/* sparsity count: number of nonzero (i,j) pairs of S over the topology */
int64_t or_pattern_nnz(const or_state *s);

#ifdef __cplusplus
}
#endif
#endif
