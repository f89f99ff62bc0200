"""Python glue for the PUFE oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain single-threaded FP64 C implementation of the assembly
(oracle.c).  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, single thread)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [
        ("lat", C.c_double * 9), ("mesh", C.c_int * 3), ("fe_order", C.c_int),
        ("n_atoms", C.c_int), ("pos", C.POINTER(C.c_double)), ("species", C.POINTER(C.c_int)),
        ("n_enr", C.c_int), ("enr_species", C.POINTER(C.c_int)), ("enr_l", C.POINTER(C.c_int)),
        ("enr_a", C.POINTER(C.c_double)), ("enr_rc", C.POINTER(C.c_double)),
        ("enr_re", C.POINTER(C.c_double)),
        ("q_n", C.c_int), ("q_nref", C.c_int), ("q_levels", C.c_int), ("q_mode", C.c_int),
        ("q_dist", C.c_double), ("q_tol", C.c_double),
        ("enr_nrad", C.POINTER(C.c_int)), ("enr_rad", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.or_setup.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_void_p)]
        L.or_setup.restype = C.c_int
        L.or_free.argtypes = [C.c_void_p]
        L.or_sizes.argtypes = [C.c_void_p, _i64p]
        L.or_dof_offset.argtypes = [C.c_void_p, _i64p]
        L.or_vertex_functions.argtypes = [C.c_void_p, C.c_int64, _i32p]
        L.or_vertex_functions.restype = C.c_int
        L.or_quadrature.argtypes = [C.c_void_p, _f64p, _f64p, _i64p]
        L.or_leaves.argtypes = [C.c_void_p, _i32p, _i32p, _i64p]
        L.or_element_nloc.argtypes = [C.c_void_p, C.c_int64]
        L.or_element_nloc.restype = C.c_int
        L.or_element_dofs.argtypes = [C.c_void_p, C.c_int64, _i64p, _i32p]
        L.or_element_matrices.argtypes = [C.c_void_p, C.c_int64, _f64p, _f64p, _f64p]
        L.or_assemble_dense.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p]
        L.or_assemble_block.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int64, C.c_int64,
                                        _f64p, _f64p]
        L.or_backward_dense.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, C.c_void_p,
                                        _f64p, _f64p]
        L.or_backward_element.argtypes = [C.c_void_p, C.c_int64, _f64p, _f64p, _f64p, C.c_void_p,
                                          _f64p, _f64p]
        L.or_set_positions.argtypes = [C.c_void_p, _f64p]
        L.or_basis_at.argtypes = [C.c_void_p, C.c_int64, _f64p, _f64p, _f64p]
        L.or_enrichment.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _f64p,
                                    _f64p, _f64p, _f64p]
        L.or_enrichment_bloch.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _f64p, _f64p,
                                          _f64p, _f64p]
        L.or_element_matrices_bloch.argtypes = [C.c_void_p, C.c_int64, _f64p, _f64p, _f64p, _f64p]
        L.or_assemble_dense_bloch.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p]
        L.or_assemble_block_bloch.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int64, C.c_int64,
                                              _f64p, _f64p]
        L.or_n_fe_dof.argtypes = [C.c_void_p]
        L.or_n_fe_dof.restype = C.c_int64
        L.or_fe_load.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_fe_eval.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_fe_stiffness.argtypes = [C.c_void_p, _f64p]
        L.or_lda.argtypes = [C.c_int64, _f64p, _f64p, C.c_void_p]
        L.or_gauss_legendre.argtypes = [C.c_int, _f64p, _f64p]
        L.or_lagrange.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
        L.or_solid_harmonic.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p, _f64p]
        L.or_nonlocal_f.argtypes = [C.c_void_p, _f64p, C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_void_p]
        L.or_nonlocal_f.restype = C.c_int
        L.or_nonlocal_dense.argtypes = [C.c_void_p, _f64p, C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
        L.or_nonlocal_f_bloch.argtypes = L.or_nonlocal_f.argtypes
        L.or_nonlocal_f_bloch.restype = C.c_int
        L.or_nonlocal_dense_bloch.argtypes = L.or_nonlocal_dense.argtypes
        L.or_pattern_nnz.argtypes = [C.c_void_p]
        L.or_pattern_nnz.restype = C.c_int64
        _lib = L
    return _lib


MODES = {"geom": 0, "error": 1}


class Oracle:
    """One problem set up in the oracle: DOF map, enriched sets, rule."""

    def __init__(self, prob: dict):
        L = lib()
        self.prob = prob
        self._keep = []
        p = _Problem()
        lat = np.asarray(prob["lattice"], np.float64).reshape(9)
        for i in range(9):
            p.lat[i] = lat[i]
        for d in range(3):
            p.mesh[d] = int(prob["mesh"][d])
        p.fe_order = int(prob["fe_order"])
        pos = np.ascontiguousarray(np.asarray(prob["atoms"], np.float64).reshape(-1))
        spc = np.ascontiguousarray(np.asarray(prob["species"], np.int32))
        enr = prob["enrichments"]
        es = np.array([e["species"] for e in enr] + [0], np.int32)
        el = np.array([e["l"] for e in enr] + [0], np.int32)
        ea = np.array([e["a"] for e in enr] + [0], np.float64)
        erc = np.array([e["rc"] for e in enr] + [0], np.float64)
        ere = np.array([e["re"] for e in enr] + [0], np.float64)
        enr_rad = [np.asarray(e.get("radial", ()), np.float64).reshape(-1) for e in enr]
        enr_n = np.array([len(r) for r in enr_rad] + [0], np.int32)
        rad = np.ascontiguousarray(np.concatenate(enr_rad + [np.zeros(1)]))
        self._keep += [pos, spc, es, el, ea, erc, ere, enr_n, rad]
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        p.n_atoms = len(prob["species"])
        p.pos = pos.ctypes.data_as(dp)
        p.species = spc.ctypes.data_as(ip)
        p.n_enr = len(enr)
        p.enr_species = es.ctypes.data_as(ip)
        p.enr_l = el.ctypes.data_as(ip)
        p.enr_a = ea.ctypes.data_as(dp)
        p.enr_rc = erc.ctypes.data_as(dp)
        p.enr_re = ere.ctypes.data_as(dp)
        p.enr_nrad = enr_n.ctypes.data_as(ip)
        p.enr_rad = rad.ctypes.data_as(dp)
        q = prob["quad"]
        p.q_n, p.q_nref, p.q_levels = int(q["n"]), int(q["n_ref"]), int(q["levels"])
        p.q_mode = MODES[q.get("mode", "geom")]
        p.q_dist, p.q_tol = float(q["dist"]), float(q["tol"])
        h = C.c_void_p()
        rc = L.or_setup(C.byref(p), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle setup rejected the problem (code {rc})")
        self.h = h
        sz = np.zeros(7, np.int64)
        L.or_sizes(h, sz)
        (self.n_elem, self.n_vertex, self.n_dof, self.n_qp, self.n_fe_slots,
         self.max_nloc, self.n_leaves) = map(int, sz)
        self.n_atoms = p.n_atoms

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_free(self.h)
                self.h = None
        except Exception:
            pass

    # ---- layout / rule
    def dof_offset(self):
        out = np.zeros(self.n_vertex + 1, np.int64)
        lib().or_dof_offset(self.h, out)
        return out

    def vertex_functions(self, v):
        out = np.zeros(3 * (self.max_nloc + 1), np.int32)
        n = lib().or_vertex_functions(self.h, v, out)
        return out[:3 * n].reshape(n, 3)

    def quadrature(self):
        xyz = np.zeros((self.n_qp, 3))
        w = np.zeros(self.n_qp)
        off = np.zeros(self.n_elem + 1, np.int64)
        lib().or_quadrature(self.h, xyz, w, off)
        return xyz, w, off

    def leaves(self):
        lev = np.zeros(max(self.n_leaves, 1), np.int32)
        ijk = np.zeros(3 * max(self.n_leaves, 1), np.int32)
        off = np.zeros(self.n_elem + 1, np.int64)
        lib().or_leaves(self.h, lev, ijk, off)
        return lev[:self.n_leaves], ijk[:3 * self.n_leaves].reshape(-1, 3), off

    def element_dofs(self, e):
        n = lib().or_element_nloc(self.h, e)
        g = np.zeros(n, np.int64)
        sh = np.zeros(3 * n, np.int32)
        lib().or_element_dofs(self.h, e, g, sh)
        return g, sh.reshape(n, 3)

    # ---- matrices
    def element_matrices(self, e, V_elem):
        n = lib().or_element_nloc(self.h, e)
        He = np.zeros((n, n))
        Se = np.zeros((n, n))
        lib().or_element_matrices(self.h, e, np.ascontiguousarray(V_elem, np.float64), He, Se)
        return He, Se

    def assemble_dense(self, V, kappa=(0.0, 0.0, 0.0)):
        N = self.n_dof
        H = np.zeros((N, N, 2))
        S = np.zeros((N, N, 2))
        lib().or_assemble_dense(self.h, np.ascontiguousarray(V, np.float64),
                                np.asarray(kappa, np.float64), H, S)
        return H[..., 0] + 1j * H[..., 1], S[..., 0] + 1j * S[..., 1]

    def assemble_block(self, V, kappa, v, w):
        off = self.dof_offset()
        nr, nc = off[v + 1] - off[v], off[w + 1] - off[w]
        Hb = np.zeros((nr, nc, 2))
        Sb = np.zeros((nr, nc, 2))
        lib().or_assemble_block(self.h, np.ascontiguousarray(V, np.float64),
                                np.asarray(kappa, np.float64), v, w, Hb, Sb)
        return Hb[..., 0] + 1j * Hb[..., 1], Sb[..., 0] + 1j * Sb[..., 1]

    def backward_dense(self, V, kappa, P, Q=None):
        N = self.n_dof
        Pr = np.ascontiguousarray(np.stack([P.real, P.imag], -1))
        Qr = None if Q is None else np.ascontiguousarray(np.stack([Q.real, Q.imag], -1))
        dV = np.zeros(self.n_qp)
        dR = np.zeros(3 * self.n_atoms)
        lib().or_backward_dense(self.h, np.ascontiguousarray(V, np.float64),
                                np.asarray(kappa, np.float64), Pr,
                                None if Qr is None else Qr.ctypes.data, dV, dR)
        return dV, dR.reshape(-1, 3)

    def backward_element(self, e, V_elem, kappa, Ploc, Qloc=None):
        """Adjoint contribution of element e from the entries P[g_a][g_b] of its
        local functions (n x n complex)."""
        n = Ploc.shape[0]
        Pr = np.ascontiguousarray(np.stack([Ploc.real, Ploc.imag], -1))
        Qr = None if Qloc is None else np.ascontiguousarray(np.stack([Qloc.real, Qloc.imag], -1))
        nq = len(V_elem)
        dV = np.zeros(nq)
        dR = np.zeros(3 * self.n_atoms)
        lib().or_backward_element(self.h, e, np.ascontiguousarray(V_elem, np.float64),
                                  np.asarray(kappa, np.float64), Pr,
                                  None if Qr is None else Qr.ctypes.data, dV, dR)
        return dV, dR.reshape(-1, 3)

    def set_positions(self, pos):
        lib().or_set_positions(self.h, np.ascontiguousarray(np.asarray(pos, np.float64).reshape(-1)))

    def basis_at(self, e, xi):
        n = lib().or_element_nloc(self.h, e)
        val = np.zeros(n)
        grad = np.zeros(3 * n)
        lib().or_basis_at(self.h, e, np.asarray(xi, np.float64), val, grad)
        return val, grad.reshape(n, 3)

    def enrichment(self, atom, desc, m, x):
        v = np.zeros(1)
        g = np.zeros(3)
        h = np.zeros(9)
        lib().or_enrichment(self.h, atom, desc, m, np.asarray(x, np.float64), v, g, h)
        return v[0], g, h.reshape(3, 3)

    # ---- Bloch-periodic enrichment (f(R) = exp(i k.R) in eq. Psi, periodic PU)
    def enrichment_bloch(self, atom, desc, m, x, kappa):
        """Psi^k and its gradient at x (complex)."""
        v = np.zeros(2)
        g = np.zeros(6)
        lib().or_enrichment_bloch(self.h, atom, desc, m, np.asarray(x, np.float64),
                                  np.asarray(kappa, np.float64), v, g)
        return v[0] + 1j * v[1], g[:3] + 1j * g[3:]

    def element_matrices_bloch(self, e, V_elem, kappa):
        n = lib().or_element_nloc(self.h, e)
        He = np.zeros((n, n, 2))
        Se = np.zeros((n, n, 2))
        lib().or_element_matrices_bloch(self.h, e, np.ascontiguousarray(V_elem, np.float64),
                                        np.asarray(kappa, np.float64), He, Se)
        return He[..., 0] + 1j * He[..., 1], Se[..., 0] + 1j * Se[..., 1]

    def assemble_dense_bloch(self, V, kappa):
        N = self.n_dof
        H = np.zeros((N, N, 2))
        S = np.zeros((N, N, 2))
        lib().or_assemble_dense_bloch(self.h, np.ascontiguousarray(V, np.float64),
                                      np.asarray(kappa, np.float64), H, S)
        return H[..., 0] + 1j * H[..., 1], S[..., 0] + 1j * S[..., 1]

    def assemble_block_bloch(self, V, kappa, v, w):
        off = self.dof_offset()
        nr, nc = off[v + 1] - off[v], off[w + 1] - off[w]
        Hb = np.zeros((nr, nc, 2))
        Sb = np.zeros((nr, nc, 2))
        lib().or_assemble_block_bloch(self.h, np.ascontiguousarray(V, np.float64),
                                      np.asarray(kappa, np.float64), v, w, Hb, Sb)
        return Hb[..., 0] + 1j * Hb[..., 1], Sb[..., 0] + 1j * Sb[..., 1]

    def assemble(self, V, kappa):
        """Dense H, S in the problem's enrichment form ("enrichment_phase":
        "periodic", the default, or "bloch")."""
        if self.prob.get("enrichment_phase", "periodic") == "bloch":
            return self.assemble_dense_bloch(V, kappa)
        return self.assemble_dense(V, kappa)

    # ---- self-consistent field pieces (section "Self-consistent calculations")
    @property
    def n_fe_dof(self):
        return int(lib().or_n_fe_dof(self.h))

    def fe_load(self, f):
        """b_i = sum_q w_q phi_i(x_q) f_q over the classical FE functions."""
        b = np.zeros(self.n_fe_dof)
        lib().or_fe_load(self.h, np.ascontiguousarray(f, np.float64), b)
        return b

    def fe_eval(self, u):
        """sum_i u_i phi_i at every point of the rule."""
        out = np.zeros(self.n_qp)
        lib().or_fe_eval(self.h, np.ascontiguousarray(u, np.float64), out)
        return out

    def fe_stiffness(self):
        N = self.n_fe_dof
        K = np.zeros((N, N))
        lib().or_fe_stiffness(self.h, K)
        return K

    def hartree(self, n_qp):
        """V_H at the rule's points for the electron density n (eq. poisson
        for the electrons' part of the charge, whose ionic part the local
        ionic potential carries): find v in the classical FE space with
        int grad phi_i . grad V_H = 4 pi int phi_i (n - nbar), nbar = int n /
        volume (the neutralising background), and int V_H = 0; a dense solve
        of the bordered system [K m; m^T 0], m_i = int phi_i.  Returns
        (V_H at the points, v)."""
        _, w, _ = self.quadrature()
        b = self.fe_load(n_qp)
        m = self.fe_load(np.ones(self.n_qp))
        nbar = float(np.dot(w, n_qp)) / float(np.sum(w))
        K = self.fe_stiffness()
        N = K.shape[0]
        A = np.zeros((N + 1, N + 1))
        A[:N, :N] = K
        A[:N, N] = m
        A[N, :N] = m
        rhs = np.concatenate([4.0 * np.pi * (b - nbar * m), [0.0]])
        v = np.linalg.solve(A, rhs)[:N]
        return self.fe_eval(v), v

    def _projectors(self, projectors):
        pr = list(projectors if projectors is not None else self.prob.get("projectors", []))
        sp = np.array([q["species"] for q in pr] + [0], np.int32)
        ll = np.array([q["l"] for q in pr] + [0], np.int32)
        aa = np.array([q["a"] for q in pr] + [0], np.float64)
        rc = np.array([q["rc"] for q in pr] + [0], np.float64)
        hh = np.array([q["h"] for q in pr] + [0], np.float64)
        return len(pr), sp, ll, aa, rc, hh

    def nonlocal_f(self, kappa=(0.0, 0.0, 0.0), projectors=None, bloch=False):
        """f_J^i of the separable nonlocal term (n_fun x N complex), over the
        basis of the periodic or (bloch) the Bloch-periodic enrichment."""
        n, sp, ll, aa, rc, _ = self._projectors(projectors)
        k = np.asarray(kappa, np.float64)
        fn = lib().or_nonlocal_f_bloch if bloch else lib().or_nonlocal_f
        nf = fn(self.h, k, n, sp, ll, aa, rc, None)
        F = np.zeros((max(nf, 1), self.n_dof, 2))
        fn(self.h, k, n, sp, ll, aa, rc, F.ctypes.data)
        return (F[..., 0] + 1j * F[..., 1])[:nf]

    def nonlocal_dense(self, kappa=(0.0, 0.0, 0.0), projectors=None, bloch=False):
        """The N x N separable nonlocal term sum_J h_J f_J^i conj(f_J^j)."""
        n, sp, ll, aa, rc, hh = self._projectors(projectors)
        N = self.n_dof
        Vn = np.zeros((N, N, 2))
        fn = lib().or_nonlocal_dense_bloch if bloch else lib().or_nonlocal_dense
        fn(self.h, np.asarray(kappa, np.float64), n, sp, ll, aa, rc, hh, Vn)
        return Vn[..., 0] + 1j * Vn[..., 1]

    def pattern_nnz(self):
        return int(lib().or_pattern_nnz(self.h))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().or_gauss_legendre(n, x, w)
    return x, w


def lagrange(p, j, t):
    v = C.c_double()
    d = C.c_double()
    lib().or_lagrange(p, j, float(t), C.byref(v), C.byref(d))
    return v.value, d.value


def solid_harmonic(l, m, r):
    v = np.zeros(1)
    g = np.zeros(3)
    h = np.zeros(9)
    lib().or_solid_harmonic(l, m, np.asarray(r, np.float64), v, g, h)
    return v[0], g, h.reshape(3, 3)


def generalized_eigh(H, S, m):
    """Lowest m eigenvalues of H c = eps S c (dense LAPACK through scipy), the
    discrete generalized eigenproblem of eq. disceig3d."""
    import scipy.linalg as sl
    return sl.eigh(H, S, eigvals_only=True, subset_by_index=[0, m - 1])


def potential_np(xyz, prob):
    """V at the oracle's points through the shared input generator."""
    import torch
    from workloads.potential import potential_at
    return potential_at(torch.from_numpy(np.ascontiguousarray(xyz)), prob).numpy()


def lda(rho):
    """LDA exchange-correlation potential and energy per electron at the
    electron densities rho (or_lda)."""
    rho = np.ascontiguousarray(rho, np.float64)
    v = np.zeros_like(rho)
    e = np.zeros_like(rho)
    lib().or_lda(rho.size, rho, v, e.ctypes.data)
    return v, e


def fermi_level(eps, n_el, sigma, weights):
    """Chemical potential mu with sum_k weights[k] sum_i 2 f((eps[k][i] - mu) /
    sigma) = n_el, f(x) = 1 / (1 + e^x) (Fermi-Dirac smearing of width sigma),
    by 200 bisection steps on [min eps - 40 sigma, max eps + 40 sigma]; returns
    mu and the occupations (weights included) per k-point."""
    def occ(mu):
        return [wk * (1.0 - np.tanh((e - mu) / (2.0 * sigma))) for e, wk in zip(eps, weights)]

    lo = min(float(e.min()) for e in eps) - 40.0 * sigma
    hi = max(float(e.max()) for e in eps) + 40.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(float(o.sum()) for o in occ(mid)) < n_el:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    return mu, occ(mu)


def scf(prob, n_iter, alpha=0.3, n_extra=2, smearing=None):
    """Fixed-point iteration of fig. scf on the oracle (periodic enrichment):
    from V_in = V_ion (the local ionic potential at the rule's points), per
    iteration: H, S at every k-point of prob (eq. disceig3d), the states
    occupied with weight 2 / n_k (the lowest n_el / 2 of each k-point, or with
    smearing > 0 the Fermi-Dirac occupations of fermi_level), the electron
    density n at the points from the adjoint's dL/dV with P = sum f c c^H
    (eq. rhoe), V_out = V_ion + V_H[n] + V_xc[n] (eqs. veff, poisson), and the
    linear mix V_in += alpha (V_out - V_in).  Returns V_in after n_iter
    iterations and per iteration the lowest ceil(n_el/2) + n_extra eigenvalues
    of every k-point and the residual (int (V_out - V_in)^2)^(1/2)."""
    import scipy.linalg as sl
    o = Oracle(prob)
    xyz, w, _ = o.quadrature()
    V_ion = potential_np(xyz, prob)
    n_el = sum(prob["species_info"][s]["Z"] for s in prob["species"])
    n_occ = int(np.ceil(n_el / 2 - 1e-12))
    if not smearing:
        assert abs(2 * n_occ - n_el) < 1e-12, "an even number of electrons is assumed without smearing"
    kpts = [tuple(k) for k in prob["kpts"]]
    V = V_ion.copy()
    hist = []
    for _ in range(n_iter):
        dens = np.zeros(o.n_qp)
        evs = []
        sols = []
        for kap in kpts:
            H, S = o.assemble_dense(V, kap)
            eps, Cv = sl.eigh(H, S)
            evs.append(eps[:n_occ + n_extra])
            sols.append((eps, Cv))
        if smearing:
            _, occ = fermi_level([e for e, _ in sols], n_el, smearing, [1.0 / len(kpts)] * len(kpts))
        else:
            occ = [np.where(np.arange(len(e)) < n_occ, 2.0 / len(kpts), 0.0) for e, _ in sols]
        for kap, (eps, Cv), f in zip(kpts, sols, occ):
            keep = f > 1e-14 * f.max()
            Co = Cv[:, keep] * f[keep]
            Pk = Co @ Cv[:, keep].conj().T
            dV, _ = o.backward_dense(V, kap, Pk)
            dens += dV / w
        vh, _ = o.hartree(dens)
        vxc, _ = lda(dens)
        Vout = V_ion + vh + vxc
        hist.append((np.array(evs), float(np.sqrt(np.dot(w, (Vout - V) ** 2)))))
        V = V + alpha * (Vout - V)
    return V, hist
