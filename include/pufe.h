/*
 * pufe.h -- C ABI of the MI355X (gfx950) PUFE Hamiltonian/overlap assembly.
 *
 * Method: Pask & Sukumar, "Partition of unity finite element method for
 * quantum mechanical materials calculations".  The library discretises the
 * Kohn-Sham eigenproblem of a periodic cell in the PUFE basis (eq. pufebasis):
 * classical C0 finite elements plus trilinear partition-of-unity functions
 * times atom-centred enrichment functions R(r) Y_lm summed over lattice images
 * (eqs. Psitilde, Psi), under Bloch boundary conditions (eqs. bloch,
 * wbpspace), and assembles the sparse Hermitian matrices of the generalized
 * eigenproblem H c = eps S c (eq. disceig3d):
 *     H_ij = int 1/2 grad phi_i^* . grad phi_j + phi_i^* V phi_j,
 *     S_ij = int phi_i^* phi_j,
 * with the per-element adaptive quadrature rule of section "Adaptive
 * quadrature".  The local potential V is an input given at the quadrature
 * points.  The FE and PU functions carry the Bloch phase at the cell boundary
 * and the enrichment is periodic (section "Self-consistent calculations"), so
 * every element matrix is real and one contraction serves all k-points.  The
 * Bloch-periodic enrichment of eq. Psi is the alternative form
 * (pufe_set_enrichment_phase).
 *
 * Conventions
 *  - Every call returns int: PUFE_OK (0) or a negative PUFE_ERR_* code;
 *    pufe_last_error_message() gives the detail.  No exception crosses the ABI.
 *  - Units: bohr and hartree.  k-points are reduced coordinates kappa
 *    (k = sum_i kappa_i b_i, b_i . a_j = 2 pi delta_ij); a function whose node
 *    wraps across the cell boundary by the lattice shift n carries the phase
 *    exp(2 pi i kappa . n).
 *  - Positions are Cartesian double[n][3]; the lattice is double[3][3], rows
 *    a_1, a_2, a_3, right-handed.  Complex values are interleaved (re, im).
 *  - Pointers named d_* are device (HIP) pointers on the context's device;
 *    all others are host pointers.  The caller owns every buffer it passes;
 *    no call keeps a caller pointer after it returns.  The library owns only
 *    its context-internal tables and workspace, freed by pufe_destroy().
 *  - Streams are hipStream_t passed as void* (NULL = default stream).  Device
 *    work is enqueued asynchronously on that stream.  pufe_setup, pufe_query,
 *    pufe_get_layout and pufe_get_leaves are synchronous.
 *  - Calls on one context are not thread-safe.
 *
 * Canonical orders (fixed so that callers can build inputs)
 *  - Elements and vertices: id = (i3 n2 + i2) n1 + i1.
 *  - DOFs, vertex-major: for vertex v the FE slots (trilinear: 1; triquadratic:
 *    8, slot s1 + 2 s2 + 4 s3 where s_d = 1 is the +1/2 midpoint; serendipity:
 *    7, slot 0 the vertex and 1 + 2 d + t the node at 1/3 (t = 0) or 2/3
 *    (t = 1) of its positive edge along d), then v's enriched functions
 *    ordered by atom, descriptor, m = -l..l.
 *  - Quadrature points: element-major; inside an element the octree leaves
 *    depth first (children c = c1 + 2 c2 + 4 c3); inside a leaf the n^3 Gauss
 *    points with the first reference index fastest.
 *  - H and S are returned as variable-block BSR keyed by vertex (see
 *    pufe_get_layout), full storage (both triangles).
 */
#ifndef PUFE_H
#define PUFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PUFE_OK 0
#define PUFE_ERR_INVALID_ARG (-1)
#define PUFE_ERR_UNSUPPORTED (-2)
#define PUFE_ERR_OOM (-3)
#define PUFE_ERR_HIP (-4)
#define PUFE_ERR_STATE (-5)

/* precision of the element contractions */
#define PUFE_PREC_FP64 0    /* FP64 MFMA */
#define PUFE_PREC_BF16X3 1  /* 2-limb bf16 split, 3 products, FP32 MFMA accumulation */
#define PUFE_PREC_BF16X6 2  /* 3-limb bf16 split, 6 products, FP32 MFMA accumulation */

/* storage type of the assembled H and S values */
#define PUFE_OUT_C128 0     /* complex double (re, im) */
#define PUFE_OUT_C64 1      /* complex float (re, im) */
#define PUFE_OUT_F64_GAMMA 2 /* real double; every k-point must be 0 (Gamma) */

/* quadrature refinement modes (section "Adaptive quadrature") */
#define PUFE_QUAD_GEOM 0    /* split a cell while it lies within `dist` of a nucleus image */
#define PUFE_QUAD_ERROR 1   /* the paper's rule: split while |Q_n - Q_ref| > tol for Psi^2 or |grad Psi|^2 */

/* form of the enrichment functions, f(R) in eq. Psi */
#define PUFE_ENR_PERIODIC 0 /* f(R) = 1; FE and PU functions carry the boundary phase (the default) */
#define PUFE_ENR_BLOCH 1    /* f(R) = exp(i k.R); PU functions periodic, FE functions carry the phase */

typedef struct pufe_ctx pufe_ctx;

/* One enrichment descriptor: the 2l+1 functions R(r) Y_lm(r_hat), real
 * orthonormal Y_lm without Condon-Shortley phase, centred on every atom of
 * `species` and summed over lattice images (eqs. Psitilde, Psi with
 * f(R) = 1).  A vertex carries them iff its minimum-image distance to the
 * atom is below re (section "Partition of unity enrichment functions").
 * The radial R (zero for r >= rc):
 *   kind 0 (analytic):  R(r) = r^l exp(-a r^2) (1 - (r/rc)^2)^3;
 *   kind 1 (tabulated, the paper's form): R(r) = r^l u(r), u the cubic spline
 *     fit of the pseudoatomic radial times the C^3 cutoff
 *     h(r, rc) = 1 + 20 x^7 - 70 x^6 + 84 x^5 - 35 x^4 (x = r/rc): radial[j],
 *     j = 0 .. n_radial-1, are samples of the pseudoatomic radial divided by
 *     r^l at r_j = j rc/(n_radial-1); u interpolates radial[j] h(r_j, rc) with
 *     end slopes u'(0) = 0 and u'(rc) = 0.  `a` is not used.
 * The samples are copied by pufe_set_problem (caller-owned host memory). */
typedef struct {
    int species;
    int l;            /* 0..3 */
    int radial_kind;  /* 0 analytic, 1 tabulated */
    double a;         /* kind 0: Gaussian exponent, > 0 */
    double rc;        /* cutoff radius, > 0 */
    double re;        /* support radius, >= 0 */
    const double *radial;  /* kind 1: n_radial finite samples (host), else NULL */
    int n_radial;          /* kind 1: 4 .. 4096 */
} pufe_enrichment;

/* One projector descriptor of the separable nonlocal potential (eq.
 * disceig3d): the 2l+1 projector functions
 *   v_lm(r) = exp(-a r^2) (1 - (r/rc)^2)^3 r^l Y_lm(r_hat)   (r < rc, zero beyond)
 * centred on every atom of `species`, with weight h (hartree): H gains
 *   sum_J h f_J^i conj(f_J^j),  f_J^i = int phi_i^* sum_n exp(i k . a_n) v_J(x - tau - a_n) dx.
 * (The radial form stands in for the tabulated projectors of a separable
 * pseudopotential.) */
typedef struct {
    int species;
    int l;            /* 0..3 */
    double a;         /* Gaussian exponent, > 0 */
    double rc;        /* cutoff radius, > 0 */
    double h;         /* weight (hartree) */
} pufe_projector;

/* The per-element rule (section "Adaptive quadrature"): leaves of an octree
 * over the reference cube, each carrying the n_gauss^3 tensor Gauss rule. */
typedef struct {
    int n_gauss;      /* 1..12 */
    int n_ref;        /* reference order of the error mode, > n_gauss */
    int max_level;    /* 0..8 */
    int mode;         /* PUFE_QUAD_GEOM or PUFE_QUAD_ERROR */
    double dist;      /* GEOM: refinement distance (bohr) */
    double tol;       /* ERROR: absolute tolerance */
} pufe_quad;

typedef struct {
    int64_t n_elem, n_vertex, n_dof, n_fe_dof, n_enr_dof;
    int64_t nnzb;     /* BSR blocks */
    int64_t nnz;      /* stored complex entries of one matrix for one k-point */
    int64_t n_qp;     /* quadrature points (0 before pufe_setup) */
    int64_t n_leaves; /* octree leaves (0 before pufe_setup) */
    int32_t max_nloc; /* largest number of functions on one element (rows of its contraction: with the
                         Bloch-periodic enrichment, real and imaginary parts counted apart) */
    int32_t n_colors; /* element colours of the atomic-free scatter */
    int32_t n_atoms;
    int32_t n_fe_slots;
} pufe_sizes;

const char *pufe_error_string(int code);
/* Detail of the last error on ctx (static string if ctx is NULL). */
const char *pufe_last_error_message(const pufe_ctx *ctx);

/* Create a context bound to HIP device `device`.  No device call is made
 * until pufe_setup. */
int pufe_create(pufe_ctx **out, int device);
int pufe_destroy(pufe_ctx *ctx);

/* Define the problem (host only, no HIP call): cell (eq. bloch: lattice rows
 * a_1..a_3), mesh of n1 x n2 x n3 parallelepiped elements (each n_d >= 2),
 * classical FE order (1 = 8-node trilinear, 2 = 27-node triquadratic
 * Lagrange, 3 = 32-node cubic serendipity, the paper's choice in section
 * "Self-consistent calculations"), atoms (Cartesian positions and species),
 * enrichment descriptors
 * and the quadrature rule.  Builds the DOF map, the enriched sets, the BSR
 * layout and the element colouring.  Errors: PUFE_ERR_INVALID_ARG (null
 * pointers, non-positive volume, fe_order outside 1..3, l outside 0..3,
 * a <= 0, rc <= 0, n_d < 2),
 * PUFE_ERR_UNSUPPORTED (GEOM refinement of a non-orthorhombic cell, more
 * functions on one element than the kernels hold). */
int pufe_set_problem(pufe_ctx *ctx, const double lattice[9], const int mesh[3], int fe_order,
                     int n_atoms, const double *pos, const int *species, int n_enr,
                     const pufe_enrichment *enr, const pufe_quad *quad);

/* Add the separable nonlocal term of eq. disceig3d to H (host only; after
 * pufe_set_problem, before pufe_setup; n = 0 removes it).  The BSR pattern of
 * H and S then also couples every pair of vertices whose functions reach one
 * projector image (pufe_get_layout reports it), and every assembly adds
 * sum_J h_J f_J^i conj(f_J^j) to H at each k-point: f from the basis values
 * and projector values at the quadrature points on FP64 MFMAs (for every
 * precision of the contraction), gathered per DOF with the Bloch phases of the
 * projector images and of the basis functions.  Projector centres stay at the
 * positions given to pufe_set_problem.  Errors: PUFE_ERR_STATE after
 * pufe_setup or before pufe_set_problem, PUFE_ERR_INVALID_ARG (l outside 0..3,
 * a <= 0, rc <= 0, n < 0), PUFE_ERR_UNSUPPORTED (more than 64 projector
 * columns reach one element). */
int pufe_set_projectors(pufe_ctx *ctx, int n, const pufe_projector *proj);

/* Choose the form of the enrichment functions (eq. Psi; host only, after
 * pufe_set_problem, before pufe_setup).  PUFE_ENR_PERIODIC (the default):
 * f(R) = 1 with Bloch-periodic FE and PU functions; every element matrix is
 * real and serves all k-points.  PUFE_ENR_BLOCH: f(R) = exp(i k.R), i.e.
 *   Psi^k(x) = sum_n exp(2 pi i kappa.n) Psi~(x - tau - n.a)
 * with tau the atom position as given (moving an atom by a lattice vector
 * multiplies its functions by a constant phase), periodic PU functions and
 * Bloch-periodic classical FE functions.  The enriched functions are then
 * complex and depend on the k-point, so each assembly contracts every element
 * once per k-point: each enriched function contributes a real row (images
 * weighted by cos 2 pi kappa.n) and an imaginary row (sin), the real MFMA
 * contraction gives the Gram matrix of both, and the scatter forms the
 * complex element matrix conj(phi_a) phi_b from it.  The layout, the
 * quadrature rule (built from the periodic functions in the error-driven
 * mode) and the output types are those of the periodic form; the split
 * precisions apply as well.  The imaginary parts double an element's
 * enrichment functions and groups, so an element may be reached by at most
 * 32 enrichment functions (2l+1 per (atom, descriptor) group) in at most 16
 * groups, and hold at most 512 rows in all (FE functions plus twice its
 * enriched local functions).  The separable nonlocal term (pufe_set_projectors)
 * follows the form: its projector coefficients come from the same real and
 * imaginary rows, per k-point.  With this form pufe_assemble_backward,
 * pufe_assemble_noalloc, pufe_element_matrices and the batch give
 * PUFE_ERR_UNSUPPORTED.  Errors: PUFE_ERR_STATE after pufe_setup or before
 * pufe_set_problem, PUFE_ERR_INVALID_ARG for an unknown form,
 * PUFE_ERR_UNSUPPORTED (too many functions on an element). */
int pufe_set_enrichment_phase(pufe_ctx *ctx, int form);

/* Build the adaptive rule on the device (section "Adaptive quadrature"),
 * upload the element tables and plan the contraction work.  Synchronous.
 * The rule is built once per geometry and reused by every assembly. */
int pufe_setup(pufe_ctx *ctx, void *stream);

/* Replace the quadrature rule built by pufe_setup with a given one (debug
 * and parity use: it lets two implementations of the error-driven rule of
 * section "Adaptive quadrature", whose refinement decisions can flip where an
 * error estimate sits at the tolerance, assemble on one shared rule).  Host
 * arrays in the layout of pufe_get_leaves: level[n_leaves] (0..8),
 * ijk[n_leaves*3] cell coordinates at that level, elem_leaf_offset[n_elem+1]
 * (canonical leaf order inside an element: depth first, children
 * c = c1 + 2 c2 + 4 c3).  The leaves of each element must cover its reference
 * cube exactly once.  Re-plans the work items (a batch created before must be
 * created anew).  Synchronous.  Errors: PUFE_ERR_STATE before pufe_setup,
 * PUFE_ERR_INVALID_ARG for malformed leaves. */
int pufe_set_rule(pufe_ctx *ctx, int64_t n_leaves, const int32_t *level, const int32_t *ijk,
                  const int64_t *elem_leaf_offset, void *stream);

/* Sizes (host).  Valid after pufe_set_problem; n_qp and n_leaves after setup. */
int pufe_query(pufe_ctx *ctx, pufe_sizes *out);

/* BSR layout (host arrays, caller-allocated): dof_offset[n_vertex+1],
 * brow_ptr[n_vertex+1], bcol[nnzb] (block column vertices, ascending per row),
 * bval_offset[nnzb+1] (start of each block's values, in entries).  Block
 * (v, w) is a dense row-major b_v x b_w sub-matrix, b_v = dof_offset[v+1] -
 * dof_offset[v].  Any pointer may be NULL. */
int pufe_get_layout(pufe_ctx *ctx, int64_t *dof_offset, int64_t *brow_ptr, int32_t *bcol,
                    int64_t *bval_offset);

/* Quadrature points in canonical order (device arrays, caller-allocated):
 * d_xyz[n_qp*3] Cartesian, d_w[n_qp] weights (including the Jacobian),
 * d_elem_qp_offset[n_elem+1].  Any pointer may be NULL.  The caller evaluates
 * V at these points for pufe_assemble. */
int pufe_get_quadrature(pufe_ctx *ctx, double *d_xyz, double *d_w, int64_t *d_elem_qp_offset,
                        void *stream);

/* Octree leaves (host arrays): level[n_leaves], ijk[n_leaves*3] integer cell
 * coordinates at that level, elem_leaf_offset[n_elem+1].  Synchronous. */
int pufe_get_leaves(pufe_ctx *ctx, int32_t *level, int32_t *ijk, int64_t *elem_leaf_offset);

/* Assemble H and S for n_k k-points (eq. disceig3d).  d_V[n_qp] is the local
 * potential at the quadrature points; kpts[n_k*3] host, reduced.  d_H and
 * d_S hold n_k consecutive value arrays of nnz entries each, of type
 * out_dtype; d_S may be NULL (S does not depend on V).  The scatter is
 * atomic-free (element colouring) and deterministic.  Errors:
 * PUFE_ERR_STATE before setup, PUFE_ERR_INVALID_ARG for a bad precision or
 * dtype, or F64_GAMMA with a non-zero k-point. */
int pufe_assemble(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision,
                  int out_dtype, void *d_H, void *d_S, void *stream);

/* Allocation-free form of pufe_assemble, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it): the same arguments, kernels and results
 * as pufe_assemble, but the phase table and the K-chunk partial tiles live in
 * a fixed workspace of PUFE_NOALLOC_WORKSPACE_BYTES that the library's code
 * object brings with it (each GPU holds its own copy until the process ends;
 * its address on a device is looked up by pufe_setup).  The call allocates
 * and frees nothing and records no timing events.  Every call on one GPU
 * shares that GPU's workspace: calls that overlap on one GPU (on different
 * streams or host threads) race and give wrong results.  A problem whose
 * partial tiles (4 KiB per element tile pair and K-chunk) do not fit gives
 * PUFE_ERR_UNSUPPORTED; the other errors are those of pufe_assemble. */
#define PUFE_NOALLOC_WORKSPACE_BYTES (64ull << 20)
int pufe_assemble_noalloc(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision,
                          int out_dtype, void *d_H, void *d_S, void *stream);

/* Real element matrices of element `elem` (debug/parity): d_He, d_Se device
 * arrays of max_nloc*max_nloc doubles; the leading nloc x nloc row-major
 * block is written, nloc returned through *nloc (host). */
int pufe_element_matrices(pufe_ctx *ctx, int64_t elem, const double *d_V, int precision,
                          double *d_He, double *d_Se, int32_t *nloc, void *stream);

/* Adjoint of the assembly for one k-point.  L = Re sum conj(P_ij) H_ij +
 * Re sum conj(Q_ij) S_ij with P, Q (complex double, BSR layout of H; either
 * may be NULL) gives
 *   d_dLdV[n_qp]      = w_q sum_ab Pt_ab phi_a phi_b  (the density at x_q times w_q,
 *                       eq. rhoe when P is the occupied density matrix),
 *   d_dLdR[n_atoms*3] = derivative with respect to the enrichment centres
 *                       (rule, enriched sets and V held fixed),
 * with Pt_ab = Re(p_a P_{g_a g_b} conj(p_b)).  Output pointers may be NULL.
 * precision: PUFE_PREC_FP64, or PUFE_PREC_BF16X3 / PUFE_PREC_BF16X6 for the
 * split-precision form, in which the dense product U = Pt [grad phi; phi]
 * runs on BF16 MFMAs from two or three bf16 limbs per operand with FP32 sums
 * (the rest of the adjoint stays FP64).  Elements of more than 80 local
 * functions (or whose block of Pt, rows and enrichment Hessians do not fit in
 * LDS together) run a second FP64 kernel that streams the element's block of
 * Pt through LDS in 64 x 64 blocks; with such elements the split-precision
 * forms give PUFE_ERR_UNSUPPORTED, as does an element of more than 256
 * enriched functions.  An unknown precision gives PUFE_ERR_INVALID_ARG. */
int pufe_assemble_backward(pufe_ctx *ctx, const double *d_V, const double kpt[3], const void *d_P,
                           const void *d_Q, int precision, double *d_dLdV, double *d_dLdR,
                           void *stream);

/* Move the enrichment centres to pos[n_atoms*3] (Cartesian) keeping the
 * quadrature rule, the enriched sets and the layout of the original geometry
 * (the frozen-basis derivative that pufe_assemble_backward computes).  Each
 * centre may move at most 0.25 bohr from the position given to
 * pufe_set_problem (PUFE_ERR_INVALID_ARG otherwise).  Synchronous. */
int pufe_set_positions(pufe_ctx *ctx, const double *pos);

/* ---- Self-consistent field pieces (section "Self-consistent calculations",
 * eqs. poisson, veff, rhoe).  Vectors of the classical FE space have
 * n_fe_dof = n_vertex * n_fe_slots entries, index v * n_fe_slots + slot (the
 * FE part of the canonical DOF order); the functions are periodic (no
 * boundary phase).  Point arrays follow the rule's canonical order.  The
 * electron density at the points is w_q-weighted output of
 * pufe_assemble_backward with P = sum_i f_i c_i c_i^H (d_dLdV / w). */

/* b_i = sum_q w_q phi_i(x_q) f(x_q) over the classical FE functions: d_f[n_qp],
 * d_b[n_fe_dof] (device).  Per-element sums in a fixed order, then one sum
 * per DOF over its elements in element order (deterministic).  Errors:
 * PUFE_ERR_STATE before pufe_setup, PUFE_ERR_INVALID_ARG for null pointers. */
int pufe_fe_load(pufe_ctx *ctx, const double *d_f, double *d_b, void *stream);

/* d_out[q] = sum_i d_u[i] phi_i(x_q) at every point of the rule.  Errors as
 * pufe_fe_load. */
int pufe_fe_eval(pufe_ctx *ctx, const double *d_u, double *d_out, void *stream);

/* Hartree potential of the electron density (eq. poisson for the electrons'
 * part of the charge; the local ionic potential carries the ionic part):
 * V_H in the classical FE space with
 *   int grad phi_i . grad V_H = 4 pi int phi_i (n - nbar),  int V_H = 0,
 * nbar = int n / int 1 the neutralising background.  d_n[n_qp] is the
 * electron density at the points (electrons per bohr^3), d_vh[n_qp] receives
 * V_H at the points and d_v[n_fe_dof] (may be NULL) its FE coefficients.  The
 * stiffness matrix is taken once per rule from the kinetic term of an
 * assembly at Gamma with V = 0 (its FE rows and columns, without the separable
 * term) and kept in the context; conjugate gradients from zero until the
 * residual falls below tol times the first (at most max_iter iterations; the
 * iterations and the final relative residual are returned through iters and
 * resid, either may be NULL).  Synchronous (the iteration reads its scalars
 * back).  Errors: PUFE_ERR_STATE before pufe_setup, PUFE_ERR_INVALID_ARG for
 * null pointers, tol <= 0 or max_iter < 1. */
int pufe_hartree(pufe_ctx *ctx, const double *d_n, double *d_vh, double *d_v, double tol, int max_iter,
                 int *iters, double *resid, void *stream);

/* LDA exchange-correlation of the unpolarised electron gas at n electron
 * densities d_rho (bohr^-3): d_vxc = d(n e_xc)/dn and (d_exc may be NULL) the
 * energy per electron e_xc; Slater exchange and the Perdew-Zunger (1981) fit
 * of the Ceperley-Alder correlation, zero where the density is <= 1e-30 (the
 * paper names the LDA, not its parametrisation).  Errors:
 * PUFE_ERR_INVALID_ARG for n < 0 or null pointers, PUFE_ERR_HIP for a failed
 * launch. */
int pufe_lda_xc(int64_t n, const double *d_rho, double *d_vxc, double *d_exc, void *stream);

/* Autotuner: time the contraction of this problem for candidate work-item
 * granularities (number of K-chunk items), tile-block sizes (2..4 tiles of
 * 16 rows per work item side) and stage lengths (16, 24 or 32 quadrature
 * points per LDS stage), keep the fastest and record it in the JSON
 * file cache_path (keyed by GPU architecture, precision and problem
 * signature; NULL = no cache).  A cached entry is applied without timing.
 * Synchronous; re-plans the work items of ctx. */
int pufe_tune(pufe_ctx *ctx, int precision, const char *cache_path);

/* Batched assembly over several problems (for instance one per lattice
 * constant of an equation-of-state sweep), all set up on the same device.
 * pufe_batch_assemble runs, for every problem, the assembly of pufe_assemble
 * at the same n_k k-points: persistent contraction launches whose work
 * groups pull the work items of all problems from one queue (largest first).
 * Each problem keeps the work items and the stage length of its own plan
 * (those pufe_tune chose, else the defaults); in FP64 the problems of one
 * stage length whose combined stage fits two work groups per CU share one
 * launch and the rest another, so up to two launches per stage length, plus
 * one for the items of elements of more than 80 functions.  Then one
 * atomic-free scatter launch per element colour covers all problems.  The
 * sequence is captured once into a HIP graph and replayed;
 * a call with different pointers, k-points, precision or dtype recaptures.
 * d_V, d_H, d_S are host arrays of n device pointers (d_S may be NULL).  The
 * contexts must outlive the batch.  A context that is defined, set up or
 * tuned again after pufe_batch_create makes pufe_batch_assemble return
 * PUFE_ERR_STATE before anything is launched (the batch copied the work
 * items of the plan it was created on); create a new batch instead. */
typedef struct pufe_batch pufe_batch;
int pufe_batch_create(pufe_batch **out, pufe_ctx *const *ctxs, int n);
int pufe_batch_assemble(pufe_batch *b, const double *const *d_V, const double *kpts, int n_k, int precision,
                        int out_dtype, void *const *d_H, void *const *d_S, void *stream);
int pufe_batch_destroy(pufe_batch *b);
const char *pufe_batch_last_error_message(const pufe_batch *b);

/* Expand one BSR value array (out_dtype C128 or F64_GAMMA) into a dense
 * row-major n_dof x n_dof complex double matrix d_dense (device). */
int pufe_bsr_to_dense(pufe_ctx *ctx, const void *d_bsr, int dtype, double *d_dense, void *stream);

/* Kernel timing for measurement.  When enabled, every contraction and every
 * scatter phase enqueued by pufe_assemble is bracketed by HIP events on the
 * caller's stream.  pufe_kernel_times waits for the recorded events and
 * returns the summed milliseconds and launch counts of
 *   [0] the element contraction kernel, [1] the zero-fill + coloured scatter
 *       (with the nonlocal gather and update when projectors are set),
 *   [2] the adjoint kernel(s), [3] the sum of the K-chunk partial tiles,
 *   [4] the projector-coefficient kernels of the nonlocal term,
 * clearing them when reset != 0.  out_ms[5] and counts[5] are host arrays. */
int pufe_enable_timing(pufe_ctx *ctx, int on);
int pufe_kernel_times(pufe_ctx *ctx, double *out_ms, int64_t *counts, int reset);

#ifdef __cplusplus
}
#endif
#endif
