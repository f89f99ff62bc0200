"""Pins of the oracle's self-consistent field pieces (section "Self-consistent
calculations", eqs. poisson, veff, rhoe):

- the classical FE load vector against closed-form integrals of the nodal
  functions (trilinear and triquadratic), its sum against the integral of f;
- FE evaluation against the trilinear interpolant written out in numpy;
- the FE stiffness matrix against its Kronecker-sum construction from 1D
  periodic stiffness and mass matrices (trilinear and triquadratic);
- the Hartree solve: a single Fourier mode of the density gives nodal values
  4 pi cos(k x) / k^2 exactly on trilinear elements (the discrete symbol of
  the mode cancels), zero mean, and a constant density gives zero;
- LDA: v_xc = d(n e_xc)/dn by central differences on both sides of r_s = 1,
  the Slater exchange constant at r_s = 1, continuity of the correlation fit;
- the fixed-point iteration: the density integrates to the electron count and
  the residual falls;
- Fermi-Dirac smearing: the occupations hold the electron count, a small
  width on an insulator reproduces the integer filling, and an odd electron
  count iterates with a falling residual."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W


def bare(L, mesh, p=1, n=4, levels=0):
    return {
        "lattice": [[L[0], 0, 0], [0, L[1], 0], [0, 0, L[2]]], "mesh": list(mesh), "fe_order": p,
        "atoms": [[0.3, 0.2, 0.1]], "species": [0], "species_info": [{"name": "X", "Z": 2.0, "rloc": 0.5}],
        "enrichments": [{"species": 0, "l": 0, "a": 1.0, "rc": 1.5, "re": 1.0}],
        "quad": {"n": n, "n_ref": n + 3, "levels": levels, "mode": "geom", "dist": 0.6, "tol": 1e-6},
        "kpts": [[0, 0, 0]], "n_eig": 4, "potential": {"cutoff": 12.0},
    }


def fe_coords(o, prob):
    """Cartesian position of every classical FE node (index v * nfs + slot)."""
    n = np.array(prob["mesh"])
    h = np.diag(np.array(prob["lattice"])) / n
    nfs = o.n_fe_dof // o.n_vertex
    X = np.zeros((o.n_fe_dof, 3))
    for v in range(o.n_vertex):
        j = np.array([v % n[0], (v // n[0]) % n[1], v // (n[0] * n[1])])
        for s in range(nfs):
            mid = np.array([(s >> d) & 1 for d in range(3)]) if nfs == 8 else np.zeros(3)
            X[v * nfs + s] = (j + 0.5 * mid) * h
    return X


@pytest.mark.parametrize("p", [1, 2])
def test_load_vector_closed_forms(p):
    prob = bare((3.0, 3.6, 4.2), (3, 3, 2), p=p, levels=1)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    m = o.fe_load(np.ones(o.n_qp))
    h = np.array([1.0, 1.2, 2.1])
    # 1D nodal integrals: vertex h (linear), h/3 (quadratic); midpoint 2h/3
    X = fe_coords(o, prob)
    nfs = o.n_fe_dof // o.n_vertex
    for i in range(o.n_fe_dof):
        s = i % nfs
        want = 1.0
        for d in range(3):
            mid = (s >> d) & 1 if nfs == 8 else 0
            want *= h[d] if p == 1 else (2.0 * h[d] / 3.0 if mid else h[d] / 3.0)
        assert abs(m[i] - want) < 1e-13 * want, (i, X[i])
    rng = np.random.default_rng(0)
    f = rng.normal(size=o.n_qp)
    assert abs(o.fe_load(f).sum() - np.dot(w, f)) < 1e-12 * np.abs(w * f).sum()


def test_eval_is_the_trilinear_interpolant():
    prob = bare((3.0, 3.6, 4.2), (3, 4, 2), p=1, levels=1)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    rng = np.random.default_rng(1)
    u = rng.normal(size=o.n_fe_dof)
    n = np.array(prob["mesh"])
    h = np.diag(np.array(prob["lattice"])) / n
    t = xyz / h
    j0 = np.floor(t).astype(int)
    fr = t - j0
    want = np.zeros(o.n_qp)
    for c in itertools.product((0, 1), repeat=3):
        j = (j0 + np.array(c)) % n
        wgt = np.prod(np.where(np.array(c) == 1, fr, 1.0 - fr), axis=1)
        want += wgt * u[(j[:, 2] * n[1] + j[:, 1]) * n[0] + j[:, 0]]
    assert np.abs(o.fe_eval(u) - want).max() < 1e-13


def periodic_1d(p, n, h):
    """1D periodic stiffness and mass matrices of order p on n elements of
    length h; index 2 j + s for quadratic (s = 1 the midpoint), j linear."""
    if p == 1:
        Ke = np.array([[1, -1], [-1, 1]]) / h
        Me = np.array([[2, 1], [1, 2]]) * h / 6
        idx = lambda e: [e, (e + 1) % n]  # noqa: E731
        N = n
    else:
        Ke = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h)
        Me = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) * h / 30
        idx = lambda e: [2 * e, 2 * e + 1, (2 * e + 2) % (2 * n)]  # noqa: E731
        N = 2 * n
    K, M = np.zeros((N, N)), np.zeros((N, N))
    for e in range(n):
        ii = idx(e)
        K[np.ix_(ii, ii)] += Ke
        M[np.ix_(ii, ii)] += Me
    return K, M


@pytest.mark.parametrize("p", [1, 2])
def test_stiffness_is_the_kronecker_sum(p):
    mesh = (3, 2, 4)
    prob = bare((3.0, 3.6, 4.2), mesh, p=p, levels=1)
    o = oracle.Oracle(prob)
    K = o.fe_stiffness()
    h = np.diag(np.array(prob["lattice"])) / np.array(mesh)
    one = [periodic_1d(p, mesh[d], h[d]) for d in range(3)]
    (Kx, Mx), (Ky, My), (Kz, Mz) = one
    K3 = np.kron(Kz, np.kron(My, Mx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Mz, np.kron(My, Kx))
    # permutation from the tensor index (i3, i2, i1) to v * nfs + slot
    n1, n2, n3 = mesh
    q = 1 if p == 1 else 2
    perm = np.zeros(K3.shape[0], int)
    for i3, i2, i1 in itertools.product(range(q * n3), range(q * n2), range(q * n1)):
        t = (i3 * q * n2 + i2) * q * n1 + i1
        j = (i1 // q, i2 // q, i3 // q)
        s = (i1 % q) + 2 * (i2 % q) + 4 * (i3 % q) if p == 2 else 0
        v = (j[2] * n2 + j[1]) * n1 + j[0]
        perm[t] = v * (8 if p == 2 else 1) + s
    Kp = np.zeros_like(K3)
    Kp[np.ix_(perm, perm)] = K3
    assert np.abs(K - Kp).max() < 1e-12 * np.abs(Kp).max()
    assert np.abs(K.sum(axis=1)).max() < 1e-12 * np.abs(K).max()


def test_hartree_of_a_fourier_mode():
    L = (6.0, 3.0, 3.0)
    prob = bare(L, (8, 2, 2), p=1, n=6, levels=0)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    k = 2 * np.pi / L[0]
    dens = 1.0 + 0.3 * np.cos(k * xyz[:, 0])
    vh, v = o.hartree(dens)
    X = fe_coords(o, prob)
    want = 4 * np.pi * 0.3 * np.cos(k * X[:, 0]) / k ** 2
    assert np.abs(v - want).max() < 1e-9 * np.abs(want).max()
    assert abs(np.dot(w, vh)) < 1e-12 * np.abs(w * vh).sum()
    vh0, _ = o.hartree(np.full(o.n_qp, 0.7))
    assert np.abs(vh0).max() < 1e-12


def test_lda_derivative_and_constants():
    rs = np.array([0.05, 0.3, 0.7, 0.999, 1.001, 1.5, 3.0, 8.0])
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    v, e = oracle.lda(n)
    hstep = 1e-6 * n
    _, ep = oracle.lda(n + hstep)
    _, em = oracle.lda(n - hstep)
    dfd = ((n + hstep) * ep - (n - hstep) * em) / (2 * hstep)
    assert np.abs(dfd - v).max() < 1e-7
    # Slater exchange at r_s = 1: -(3/4)(9/(4 pi^2))^(1/3)
    _, e1 = oracle.lda(np.array([3.0 / (4.0 * np.pi)]))
    _, el = oracle.lda(np.array([3.0 / (4.0 * np.pi * 0.999999 ** 3)]))
    ex1 = -0.75 * (9.0 / (4.0 * np.pi ** 2)) ** (1.0 / 3.0)
    assert abs(ex1 + 0.4581652932831429) < 1e-15
    ec_hi, ec_lo = e1[0] - ex1, el[0] - ex1 * (1 / 0.999999)
    assert abs(ec_hi - ec_lo) < 1e-4 and -0.07 < ec_hi < -0.05
    vz, ez = oracle.lda(np.array([0.0, -1.0]))
    assert np.all(vz == 0) and np.all(ez == 0)


def test_scf_density_count_and_residual():
    prob = W.small("lih", mesh=(2, 2, 2), fe_order=1, levels=1, n=3, a=4.6)
    V, hist = oracle.scf(prob, 4, alpha=0.3)
    res = [r for _, r in hist]
    assert all(b < a for a, b in zip(res, res[1:]))
    # the density of the last iteration integrates to the electron count
    o = oracle.Oracle(prob)
    _, w, _ = o.quadrature()
    import scipy.linalg as sl
    H, S = o.assemble_dense(V, (0.0, 0.0, 0.0))
    eps, Cv = sl.eigh(H, S)
    Co = Cv[:, :8]
    dV, _ = o.backward_dense(V, (0.0, 0.0, 0.0), 2.0 * Co @ Co.conj().T)
    assert abs(dV.sum() - 16.0) < 1e-10
    assert np.all(dV / w > -1e-12)


def test_fermi_smearing():
    """Fermi-Dirac occupations: they hold the electron count, a small width on
    an insulator reproduces the integer filling of the lowest states, and a
    metal-like (odd) electron count runs with smearing, its density
    integrating to that count."""
    rng = np.random.default_rng(5)
    eps = [np.sort(rng.normal(size=30)) for _ in range(3)]
    for n_el, sig in ((15.0, 0.05), (20.0, 0.01), (7.0, 0.3)):
        mu, occ = oracle.fermi_level(eps, n_el, sig, [1.0 / 3] * 3)
        assert abs(sum(o.sum() for o in occ) - n_el) < 1e-10
        assert all(np.all((o >= 0) & (o <= 2.0 / 3 + 1e-15)) for o in occ)
    prob = W.small("lih", mesh=(2, 2, 2), fe_order=1, levels=1, n=3, a=4.6)
    V0, h0 = oracle.scf(prob, 2)
    V1, h1 = oracle.scf(prob, 2, smearing=1e-3)
    assert np.abs(V1 - V0).max() < 1e-10
    pc = W.small("ceal", mesh=(2, 2, 2), fe_order=1, levels=1, n=3, a=4.4,
                 kpts=((0.0, 0.0, 0.0), (0.25, 0.25, -0.25)))
    V, h = oracle.scf(pc, 2, smearing=0.02)
    assert h[1][1] < h[0][1]
