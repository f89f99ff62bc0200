"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with
itself: each checks a closed form, a library routine, a number printed in the
paper, an exact identity of the discrete problem, or finite differences.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bare(lattice, mesh, p, n=3, enrichments=(), atoms=((0.1, 0.2, 0.3),), levels=0, kpts=((0, 0, 0),)):
    return {
        "lattice": lattice, "mesh": list(mesh), "fe_order": p,
        "atoms": [list(a) for a in atoms], "species": [0] * len(atoms),
        "species_info": [{"name": "X", "Z": 1.0, "rloc": 0.5}],
        "enrichments": list(enrichments),
        "quad": {"n": n, "n_ref": n + 3, "levels": levels, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        "kpts": [list(k) for k in kpts], "n_eig": 4, "potential": {"cutoff": 12.0},
    }


def diag(a, b, c):
    return [[a, 0, 0], [0, b, 0], [0, 0, c]]


# ----------------------------------------------------------------- 1D rules

@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 8, 10])
def test_gauss_legendre_matches_library_and_is_exact(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-14, rtol=0) and np.allclose(w, wr, atol=1e-14, rtol=0)
    for k in range(2 * n):          # exact up to degree 2n-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_lagrange_kronecker_and_partition(p):
    nodes = [-1 + 2 * k / p for k in range(p + 1)]
    for j in range(p + 1):
        for k, t in enumerate(nodes):
            assert abs(oracle.lagrange(p, j, t)[0] - (1.0 if j == k else 0.0)) < 1e-15
    for t in np.linspace(-1, 1, 13):
        vals = [oracle.lagrange(p, j, t) for j in range(p + 1)]
        assert abs(sum(v for v, _ in vals) - 1) < 1e-14
        assert abs(sum(d for _, d in vals)) < 1e-13
        for j in range(p + 1):      # derivative against a central difference
            h = 1e-6
            fd = (oracle.lagrange(p, j, t + h)[0] - oracle.lagrange(p, j, t - h)[0]) / (2 * h)
            assert abs(fd - vals[j][1]) < 1e-8


# --------------------------------------------------------- solid harmonics

def _real_ylm_scipy(l, m, polar, azim):
    """Real orthonormal Y_lm without the Condon-Shortley phase from scipy's
    complex harmonics (which carry that phase)."""
    import scipy.special as sp
    am = abs(m)
    Y = sp.sph_harm_y(l, am, polar, azim)
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2) * (-1) ** am * Y.real
    return math.sqrt(2) * (-1) ** am * Y.imag


def test_solid_harmonics_match_scipy_on_sphere():
    rng = np.random.default_rng(1)
    for _ in range(20):
        polar, azim = rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi)
        r = np.array([np.sin(polar) * np.cos(azim), np.sin(polar) * np.sin(azim), np.cos(polar)])
        for l in range(4):
            for m in range(-l, l + 1):
                v, _, _ = oracle.solid_harmonic(l, m, r)
                assert abs(v - _real_ylm_scipy(l, m, polar, azim)) < 1e-13, (l, m)


def test_solid_harmonics_orthonormal_harmonic_homogeneous():
    ct, wt = np.polynomial.legendre.leggauss(12)
    nphi = 16
    phis = 2 * np.pi * np.arange(nphi) / nphi
    fns = [(l, m) for l in range(4) for m in range(-l, l + 1)]
    G = np.zeros((len(fns), len(fns)))
    for c, w in zip(ct, wt):
        s = math.sqrt(1 - c * c)
        for ph in phis:
            r = np.array([s * math.cos(ph), s * math.sin(ph), c])
            vals = np.array([oracle.solid_harmonic(l, m, r)[0] for l, m in fns])
            G += w * (2 * np.pi / nphi) * np.outer(vals, vals)
    assert np.abs(G - np.eye(len(fns))).max() < 1e-13
    rng = np.random.default_rng(2)
    for _ in range(10):
        x = rng.normal(size=3)
        for l, m in fns:
            v, g, h = oracle.solid_harmonic(l, m, x)
            assert abs(np.trace(h)) < 1e-12                    # harmonic
            assert abs(x @ g - l * v) < 1e-12                  # Euler: degree l
            assert np.abs(h @ x - (l - 1) * g).max() < 1e-12 if l > 0 else True
            assert np.abs(h - h.T).max() < 1e-14


# -------------------------------------------------------- element matrices

def _m1(h, p):
    if p == 1:
        return h / 6 * np.array([[2, 1], [1, 2]]), 1 / h * np.array([[1, -1], [-1, 1]])
    return (h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]),
            1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]))


@pytest.mark.parametrize("p", [1, 2])
def test_element_mass_stiffness_closed_form(p):
    L = (3.0, 3.6, 4.2)
    mesh = (3, 2, 4)
    prob = bare(diag(*L), mesh, p, n=3)
    o = oracle.Oracle(prob)
    h = [L[d] / mesh[d] for d in range(3)]
    Ms, Ks = zip(*[_m1(h[d], p) for d in range(3)])
    M3 = np.kron(Ms[2], np.kron(Ms[1], Ms[0]))
    K3 = (np.kron(Ms[2], np.kron(Ms[1], Ks[0])) + np.kron(Ms[2], np.kron(Ks[1], Ms[0]))
          + np.kron(Ks[2], np.kron(Ms[1], Ms[0])))
    nq = 27
    for e in (0, 5, o.n_elem - 1):
        He, Se = o.element_matrices(e, np.zeros(nq))
        assert np.abs(Se - M3).max() < 1e-14 * max(1, np.abs(M3).max())
        assert np.abs(He - 0.5 * K3).max() < 1e-13


# ------------------------------------------------------------ empty lattice

def _eig1d(n, h, p, kappa):
    """1D Bloch-reduced generalized eigenvalues of the periodic FE chain."""
    out = []
    M, K = _m1(h, p)
    for mm in range(n):
        th = 2 * np.pi * (mm + kappa) / n
        if p == 1:
            out.append(6 * (1 - np.cos(th)) / (h * h * (2 + np.cos(th))))
        else:
            T = np.array([[1, 0], [0, 1], [np.exp(1j * th), 0]])
            Kr = T.conj().T @ K @ T
            Mr = T.conj().T @ M @ T
            import scipy.linalg as sl
            out += list(sl.eigh(Kr, Mr, eigvals_only=True))
    return np.array(out)


@pytest.mark.parametrize("p,mesh,kappa", [(1, (4, 3, 5), (0.0, 0.0, 0.0)),
                                           (1, (3, 4, 3), (0.1, -0.23, 0.37)),
                                           (2, (2, 3, 2), (0.0, 0.0, 0.0)),
                                           (2, (3, 2, 2), (0.12, -0.24, 0.37))])
def test_empty_lattice_discrete_spectrum(p, mesh, kappa):
    L = (3.0, 3.3, 2.7)
    o = oracle.Oracle(bare(diag(*L), mesh, p, n=3))
    H, S = o.assemble_dense(np.zeros(o.n_qp), kappa)
    ev = oracle.generalized_eigh(H, S, 12)
    lam = [_eig1d(mesh[d], L[d] / mesh[d], p, kappa[d]) for d in range(3)]
    allev = np.sort((lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]).ravel() / 2)
    assert np.abs(ev - allev[:12]).max() < 1e-11 * max(1, allev[11])


def test_plane_wave_interpolant_fixes_phase_sign():
    """The Bloch sum of the FE functions with coefficients exp(i k.x_node) is
    the nodal interpolant of the plane wave exp(i k.x); its mass and energy
    are tensor products of the 1D forms.  A flipped boundary phase would
    break the interpolant in the wrapped elements."""
    L = (3.0, 3.3, 2.7)
    mesh = (3, 4, 3)
    kap = np.array([0.31, -0.17, 0.42])
    o = oracle.Oracle(bare(diag(*L), mesh, 1, n=3))
    H, S = o.assemble_dense(np.zeros(o.n_qp), kap)
    c = np.zeros(o.n_dof, complex)
    for v in range(o.n_vertex):
        j = (v % mesh[0], (v // mesh[0]) % mesh[1], v // (mesh[0] * mesh[1]))
        c[v] = np.exp(2j * np.pi * sum(kap[d] * j[d] / mesh[d] for d in range(3)))
    th = [2 * np.pi * kap[d] / mesh[d] for d in range(3)]
    h = [L[d] / mesh[d] for d in range(3)]
    m1 = [mesh[d] * h[d] / 3 * (2 + np.cos(th[d])) for d in range(3)]
    k1 = [mesh[d] * 2 * (1 - np.cos(th[d])) / h[d] for d in range(3)]
    s_exact = m1[0] * m1[1] * m1[2]
    h_exact = 0.5 * (k1[0] * m1[1] * m1[2] + m1[0] * k1[1] * m1[2] + m1[0] * m1[1] * k1[2])
    assert abs(c.conj() @ S @ c - s_exact) < 1e-12 * s_exact
    assert abs(c.conj() @ H @ c - h_exact) < 1e-12 * h_exact


def test_gamma_constant_in_kernel_and_zero_eigenvalue():
    prob = W.small("lih", mesh=(3, 2, 3), fe_order=2, levels=1, n=3, a=5.0)
    o = oracle.Oracle(prob)
    H, S = o.assemble_dense(np.zeros(o.n_qp))
    one = np.zeros(o.n_dof)
    off = o.dof_offset()
    for v in range(o.n_vertex):
        one[off[v]:off[v] + o.n_fe_slots] = 1.0     # sum of all FE functions = 1
    assert np.abs(H @ one).max() < 1e-12
    ev = oracle.generalized_eigh(H, S, 2)
    assert abs(ev[0]) < 1e-10


def test_ritz_values_monotone_in_enrichment_and_bounded_below():
    """Min-max: adding basis functions never raises a Ritz value; with V = 0
    the continuum eigenvalues |k+G|^2/2 bound them from below."""
    L = 4.0
    kap = np.array([0.1, 0.2, -0.15])
    evs = []
    for re in (0.0, 1.2, 2.0, 3.5):
        enr = [] if re == 0 else [{"species": 0, "l": 0, "a": 1.5, "rc": 1.9, "re": re},
                                  {"species": 0, "l": 1, "a": 1.0, "rc": 1.9, "re": re}]
        prob = bare(diag(L, L, L), (2, 2, 2), 2, n=6, enrichments=enr, atoms=((1.1, 0.9, 1.3),),
                    levels=1)
        prob["quad"]["dist"] = 1.2
        o = oracle.Oracle(prob)
        H, S = o.assemble_dense(np.zeros(o.n_qp), kap)
        evs.append(oracle.generalized_eigh(H, S, 10))
    for a, b in zip(evs, evs[1:]):
        assert np.all(b <= a + 1e-10)
    G = np.array([(i, j, k) for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)])
    exact = np.sort(0.5 * np.sum(((G + kap) * 2 * np.pi / L) ** 2, axis=1))[:10]
    for ev in evs:
        assert np.all(ev >= exact - 1e-4)


# ---------------------------------------------------------------- identities

def test_potential_shift_adds_overlap():
    prob = W.small("one", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=4.5)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    kap = (0.2, -0.1, 0.3)
    H1, S1 = o.assemble_dense(V, kap)
    H2, S2 = o.assemble_dense(V + 0.37, kap)
    assert np.abs(H2 - (H1 + 0.37 * S1)).max() < 1e-12 * np.abs(H1).max()
    assert np.abs(S2 - S1).max() == 0.0


def test_hermitian_pd_bloch_symmetries():
    prob = W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    kap = np.array([0.12, -0.24, 0.37])
    H, S = o.assemble_dense(V, kap)
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(H).max()
    assert np.abs(S - S.conj().T).max() < 1e-15 * max(1, np.abs(S).max()) * 10
    np.linalg.cholesky(S)
    Hg, Sg = o.assemble_dense(V, kap + np.array([1, -2, 1]))
    assert np.abs(Hg - H).max() < 1e-12 * np.abs(H).max()
    Hm, Sm = o.assemble_dense(V, -kap)
    assert np.abs(Hm - H.conj()).max() < 1e-13 * np.abs(H).max()
    assert np.abs(Sm - S.conj()).max() < 1e-15 * 10


def test_translation_by_lattice_vector_and_by_element():
    prob = W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=0, n=4, a=5.0)
    kap = (0.12, -0.24, 0.37)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    H, S = o.assemble_dense(oracle.potential_np(xyz, prob), kap)
    lat = np.asarray(prob["lattice"])
    # whole lattice vector: identical matrices
    p2 = dict(prob)
    p2["atoms"] = (np.asarray(prob["atoms"]) + lat[0] - 2 * lat[2]).tolist()
    o2 = oracle.Oracle(p2)
    H2, S2 = o2.assemble_dense(oracle.potential_np(xyz, p2), kap)
    assert np.abs(H2 - H).max() < 1e-11 * np.abs(H).max()
    assert np.abs(S2 - S).max() < 1e-12
    # one element spacing: same spectrum
    p3 = dict(prob)
    p3["atoms"] = (np.asarray(prob["atoms"]) + lat[0] / prob["mesh"][0]).tolist()
    o3 = oracle.Oracle(p3)
    x3, _, _ = o3.quadrature()
    H3, S3 = o3.assemble_dense(oracle.potential_np(x3, p3), kap)
    e1 = oracle.generalized_eigh(H, S, 8)
    e3 = oracle.generalized_eigh(H3, S3, 8)
    assert np.abs(e1 - e3).max() < 1e-10 * max(1, np.abs(e1).max())


def test_rotation_invariance_of_spectrum():
    """Rotating cell and atoms together (a non-orthorhombic Cartesian frame)
    leaves the spectrum unchanged; this pins the gradient transformation and
    the l = 1 harmonics."""
    prob = W.small("one", mesh=(2, 2, 3), fe_order=2, levels=0, n=4, a=4.5, re=2.0)
    from scipy.spatial.transform import Rotation
    R = Rotation.from_euler("zyx", [0.3, -0.7, 1.1]).as_matrix()
    kap = (0.1, 0.25, -0.3)
    out = []
    for rot in (np.eye(3), R):
        p = dict(prob)
        p["lattice"] = (np.asarray(prob["lattice"]) @ rot.T).tolist()
        p["atoms"] = (np.asarray(prob["atoms"]) @ rot.T).tolist()
        o = oracle.Oracle(p)
        xyz, _, _ = o.quadrature()
        H, S = o.assemble_dense(oracle.potential_np(xyz, p), kap)
        out.append(oracle.generalized_eigh(H, S, 10))
    assert np.abs(out[0] - out[1]).max() < 1e-9 * np.abs(out[0]).max()


# -------------------------------------------------------------- enrichment

def _radial_integrals(l, a, rc):
    x, w = np.polynomial.legendre.leggauss(200)
    r = 0.5 * rc * (x + 1)
    w = 0.5 * rc * w
    R = r ** l * np.exp(-a * r * r) * (1 - (r / rc) ** 2) ** 3
    dR = (l * r ** (l - 1) if l > 0 else 0 * r) * np.exp(-a * r * r) * (1 - (r / rc) ** 2) ** 3 \
        + r ** l * np.exp(-a * r * r) * (-2 * a * r * (1 - (r / rc) ** 2) ** 3
                                         - 6 * r / rc ** 2 * (1 - (r / rc) ** 2) ** 2)
    I0 = np.sum(w * R * R * r * r)
    I1 = np.sum(w * (dR * dR + l * (l + 1) * R * R / (r * r)) * r * r)
    return I0, I1


@pytest.mark.parametrize("l,a", [(0, 1.3), (1, 0.8), (2, 1.0), (3, 0.9)])
def test_isolated_enrichment_integrals_through_pu(l, a):
    """With every vertex carrying the function, the PU sums back to Psi, so
    1^T S_aa 1 = int Psi^2 and 1^T H_aa 1 = 1/2 int |grad Psi|^2 (V = 0);
    for an isolated function these are 1D radial integrals."""
    rc, L = 2.3, 6.0
    enr = [{"species": 0, "l": l, "a": a, "rc": rc, "re": 100.0}]
    prob = bare(diag(L, L, L), (2, 2, 2), 1, n=10, enrichments=enr, atoms=((2.3, 2.9, 3.4),),
                levels=1)
    prob["quad"]["dist"] = 2.5
    o = oracle.Oracle(prob)
    H, S = o.assemble_dense(np.zeros(o.n_qp))
    off = o.dof_offset()
    I0, I1 = _radial_integrals(l, a, rc)
    for m in range(2 * l + 1):
        sel = np.zeros(o.n_dof)
        for v in range(o.n_vertex):
            sel[off[v] + 1 + m] = 1.0
        assert abs(sel @ S.real @ sel - I0) < 5e-8 * I0
        assert abs(sel @ H.real @ sel - 0.5 * I1) < 2e-7 * I1


def test_enrichment_periodic_and_derivatives():
    prob = W.small("ceal", mesh=(2, 2, 2), fe_order=1, levels=0, n=2, a=4.0, rc=2.6)
    o = oracle.Oracle(prob)
    lat = np.asarray(prob["lattice"])
    rng = np.random.default_rng(3)
    for desc in (0, 3, 6, 8):
        l = prob["enrichments"][desc]["l"]
        atom = prob["enrichments"][desc]["species"]
        for _ in range(4):
            x = rng.uniform(0, 4.0, size=3)
            m = int(rng.integers(-l, l + 1))
            v, g, h = o.enrichment(atom, desc, m, x)
            v2, g2, _ = o.enrichment(atom, desc, m, x + lat[1] - lat[2])
            assert abs(v - v2) < 1e-13 and np.abs(g - g2).max() < 1e-12
            eps = 1e-5
            for k in range(3):
                dx = np.zeros(3)
                dx[k] = eps
                vp, gp, _ = o.enrichment(atom, desc, m, x + dx)
                vm, gm, _ = o.enrichment(atom, desc, m, x - dx)
                assert abs((vp - vm) / (2 * eps) - g[k]) < 1e-7 * max(1, abs(g).max())
                assert np.abs((gp - gm) / (2 * eps) - h[:, k]).max() < 1e-6 * max(1, np.abs(h).max())


# ------------------------------------------------------------------ layout

def _table1():
    rows, added = [], None
    for line in open(os.path.join(GOLDEN, "table1_sparsity.txt")):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "added":
            added = (int(line[1]), float(line[2]), float(line[3]), int(line[4]))
        else:
            rows.append((int(line[0]), int(line[1]), float(line[2]), float(line[3])))
    return rows, added


def test_sparsity_table_of_the_paper():
    rows, added = _table1()
    for cells, mesh, re, pct in rows:
        o = oracle.Oracle(W.lih_table1(re, cells=cells, mesh=mesh))
        sp = 100.0 * (1.0 - o.pattern_nnz() / o.n_dof ** 2)
        assert round(sp, 1) == pct, (cells, mesh, re, sp)
    mesh, r0, r1, n_add = added
    n0 = oracle.Oracle(W.lih_table1(r0, mesh=mesh)).n_dof
    n1 = oracle.Oracle(W.lih_table1(r1, mesh=mesh)).n_dof
    assert n1 - n0 == n_add


# -------------------------------------------------------------- quadrature

def test_rule_weights_sum_to_volume_and_geometry():
    prob = W.small("lih", mesh=(3, 2, 3), fe_order=2, levels=2, n=3, a=5.0)
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    assert abs(w.sum() - 125.0) < 1e-12
    lev, ijk, loff = o.leaves()
    lat = np.asarray(prob["lattice"])
    atoms = np.asarray(prob["atoms"])
    mesh = prob["mesh"]

    def box_dist(e, l, c):  # sampled closest distance (an upper bound of the true one)
        i = (e % mesh[0], (e // mesh[0]) % mesh[1], e // (mesh[0] * mesh[1]))
        g = np.linspace(0, 1, 9)
        best = np.inf
        for A in atoms:
            pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
            red = (np.array(i) + (np.array(c) + pts) / 2 ** l) / np.array(mesh)
            P = red @ lat
            for sh in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
                best = min(best, np.min(np.linalg.norm(P - A - sh @ lat, axis=1)))
        return best

    n_split_checked = 0
    for e in range(o.n_elem):
        for k in range(loff[e], loff[e + 1]):
            l, c = lev[k], ijk[k]
            if l >= 1:  # parent was split: it is within reach of a nucleus
                assert box_dist(e, l - 1, c // 2) <= 1.0 + 0.2
                n_split_checked += 1
    assert n_split_checked > 0
    # qp order: Gauss points with the first index fastest inside each leaf
    n = prob["quad"]["n"]
    assert np.all(np.diff(xyz[:n, 0]) > 0)


def test_adaptive_rule_converges_to_fine_uniform_rule():
    enr = [{"species": 0, "l": 0, "a": 2.0, "rc": 1.8, "re": 1.5}]
    base = bare(diag(4.0, 4.0, 4.0), (2, 2, 2), 1, n=4, enrichments=enr, atoms=((1.3, 2.2, 1.9),))
    errs = []
    fine = dict(base, quad={"n": 8, "n_ref": 9, "levels": 2, "mode": "geom", "dist": 10.0, "tol": 0})
    of = oracle.Oracle(fine)
    Hf, Sf = of.assemble_dense(np.zeros(of.n_qp))
    for levels in (0, 1, 2):
        p = dict(base, quad={"n": 4, "n_ref": 5, "levels": levels, "mode": "geom", "dist": 1.0, "tol": 0})
        o = oracle.Oracle(p)
        H, S = o.assemble_dense(np.zeros(o.n_qp))
        errs.append(np.abs(S - Sf).max())
    assert errs[2] < errs[1] < errs[0]


def test_error_driven_rule_meets_tolerance():
    enr = [{"species": 0, "l": 0, "a": 3.0, "rc": 1.8, "re": 1.6}]
    p = bare(diag(4.0, 4.0, 4.0), (2, 2, 2), 1, n=3, enrichments=enr, atoms=((1.3, 2.2, 1.9),))
    p["quad"] = {"n": 3, "n_ref": 6, "levels": 4, "mode": "error", "dist": 0, "tol": 1e-6}
    o = oracle.Oracle(p)
    lev, _, _ = o.leaves()
    assert lev.max() >= 2
    xyz, w, _ = o.quadrature()
    assert abs(w.sum() - 64.0) < 1e-12
    # the function is isolated (rc < L/2): the rule's integral of Psi^2 must
    # meet the radial closed form within the summed per-cell tolerances
    I0, _ = _radial_integrals(0, 3.0, 1.8)
    got = sum(wq * o.enrichment(0, 0, 0, xq)[0] ** 2 for xq, wq in zip(xyz, w))
    assert abs(got - I0) < 1e-6 * len(lev)
    # and a plain base rule without refinement misses it by far more
    p0 = dict(p, quad=dict(p["quad"], levels=0))
    o0 = oracle.Oracle(p0)
    x0, w0, _ = o0.quadrature()
    got0 = sum(wq * o0.enrichment(0, 0, 0, xq)[0] ** 2 for xq, wq in zip(x0, w0))
    assert abs(got0 - I0) > 10 * abs(got - I0)


# -------------------------------------------------------------- adjoint

def _loss(o, V, kap, P, Q):
    H, S = o.assemble_dense(V, kap)
    return np.real(np.sum(P.conj() * H)) + np.real(np.sum(Q.conj() * S))


def test_backward_matches_finite_differences():
    prob = W.small("lih", mesh=(2, 2, 3), fe_order=1, levels=1, n=3, a=4.6, re=1.6, rc=2.0)
    kap = np.array([0.12, -0.24, 0.37])
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    Cf = W.adjoint_factor(o.n_dof, rank=6, seed=0)
    P = Cf @ Cf.conj().T
    Cq = W.adjoint_factor(o.n_dof, rank=3, seed=1)
    Q = Cq @ Cq.conj().T
    dV, dR = o.backward_dense(V, kap, P, Q)
    # adjoint identity for the linear V-dependence
    M0 = o.assemble_dense(np.zeros_like(V), kap)[0]
    Hv = o.assemble_dense(V, kap)[0]
    assert abs(V @ dV - np.real(np.sum(P.conj() * (Hv - M0)))) < 1e-11 * abs(V @ dV)
    # a few single-point derivatives, exact because L is linear in V
    L0 = _loss(o, V, kap, P, Q)
    for q in (0, 17, o.n_qp // 2):
        e = np.zeros_like(V)
        e[q] = 1.0
        assert abs((_loss(o, V + e, kap, P, Q) - L0) - dV[q]) < 1e-10 * max(1, abs(L0))
    # forces: central differences of L with the rule, enriched sets and V frozen
    pos = np.asarray(prob["atoms"], float)
    hstep = 1e-4
    for A in (0, 3, 6):
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[A, k] += hstep
            pm[A, k] -= hstep
            o.set_positions(pp)
            Lp = _loss(o, V, kap, P, Q)
            o.set_positions(pm)
            Lm = _loss(o, V, kap, P, Q)
            o.set_positions(pos)
            fd = (Lp - Lm) / (2 * hstep)
            assert abs(fd - dR[A, k]) < 1e-6 * max(1.0, np.abs(dR).max()), (A, k, fd, dR[A, k])
