"""Pins of the oracle's 32-node cubic serendipity elements (the paper's
classical FE, section "Self-consistent calculations"): Kronecker property at
the 32 nodes, partition of unity and exact reproduction of every cubic
polynomial (and not of x^2 y^2, which the serendipity space lacks),
reference gradients against central differences, element integrals of a
cubic against closed forms, and the O(h^6) convergence of free-electron
eigenvalues with the mesh (Ritz values of a space containing the cubics).

The local order of the 32 FE functions: the 8 corners c = c1 + 2 c2 + 4 c3,
then for each direction d the edges starting at the corners with c_d = 0 in
corner order, two nodes each (at -1/3, then +1/3)."""
import itertools

import numpy as np
import pytest

import oracle


def bare(L, mesh, p=3, n=4, kpts=((0, 0, 0),)):
    return {
        "lattice": [[L[0], 0, 0], [0, L[1], 0], [0, 0, L[2]]], "mesh": list(mesh), "fe_order": p,
        "atoms": [[0.1, 0.2, 0.3]], "species": [0], "species_info": [{"name": "X", "Z": 1.0, "rloc": 0.5}],
        "enrichments": [],
        "quad": {"n": n, "n_ref": n + 3, "levels": 0, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        "kpts": [list(k) for k in kpts], "n_eig": 4, "potential": {"cutoff": 12.0},
    }


def nodes():
    out = []
    for c in range(8):
        out.append([-1.0 + 2.0 * ((c >> d) & 1) for d in range(3)])
    for d in range(3):
        for c in range(8):
            if (c >> d) & 1:
                continue
            for t in (-1.0 / 3.0, 1.0 / 3.0):
                x = [-1.0 + 2.0 * ((c >> k) & 1) for k in range(3)]
                x[d] = t
                out.append(x)
    return np.array(out)


def test_kronecker_at_the_nodes():
    o = oracle.Oracle(bare((3.0, 3.0, 3.0), (2, 2, 2)))
    X = nodes()
    assert len(X) == 32 and o.element_dofs(0)[0].size == 32
    for b, xb in enumerate(X):
        val, _ = o.basis_at(0, xb)
        e = np.zeros(32)
        e[b] = 1.0
        assert np.abs(val - e).max() < 1e-14, b


def test_partition_of_unity_and_cubic_reproduction():
    o = oracle.Oracle(bare((3.0, 3.0, 3.0), (2, 2, 2)))
    X = nodes()
    rng = np.random.default_rng(0)
    cubic = [m for m in itertools.product(range(4), repeat=3) if sum(m) <= 3]
    assert len(cubic) == 20
    for _ in range(10):
        xi = rng.uniform(-1, 1, 3)
        val, _ = o.basis_at(0, xi)
        for m in cubic:
            f_nodes = np.prod(X ** np.array(m), axis=1)
            assert abs(val @ f_nodes - np.prod(xi ** np.array(m))) < 1e-13, m
        # x^2 y^2 lies outside the serendipity space
        assert abs(val @ (X[:, 0] ** 2 * X[:, 1] ** 2) - xi[0] ** 2 * xi[1] ** 2) > 1e-6


def test_gradients_against_central_differences():
    L, mesh = (3.0, 3.6, 2.4), (2, 3, 2)
    o = oracle.Oracle(bare(L, mesh))
    rng = np.random.default_rng(1)
    scale = np.array([2.0 * mesh[d] / L[d] for d in range(3)])   # d xi_d / d x_d
    for _ in range(5):
        xi = rng.uniform(-0.9, 0.9, 3)
        _, grad = o.basis_at(3, xi)
        h = 1e-6
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fd = (o.basis_at(3, xi + e)[0] - o.basis_at(3, xi - e)[0]) / (2 * h) * scale[d]
            assert np.abs(fd - grad[:, d]).max() < 1e-7


def test_element_integrals_of_a_cubic():
    """For f = xi_1^2 xi_2 (reproduced exactly) on an element of side h:
    c^T S_e c = det J int xi1^4 xi2^2 = det J 8/15 and
    c^T H_e c (V = 0) = 1/2 (2/h)^2 det J int (4 xi1^2 xi2^2 + xi1^4) = 1/2 (2/h)^2 det J (32/9 + 8/5);
    the sum of S_e is the element volume."""
    L, mesh = (2.4, 2.4, 2.4), (2, 2, 2)
    o = oracle.Oracle(bare(L, mesh, n=5))
    h = L[0] / mesh[0]
    detJ = (h / 2) ** 3
    He, Se = o.element_matrices(0, np.zeros(5 ** 3))
    X = nodes()
    c = X[:, 0] ** 2 * X[:, 1]
    assert abs(c @ Se @ c - detJ * 8 / 15) < 1e-13
    assert abs(c @ He @ c - 0.5 * (2 / h) ** 2 * detJ * (32 / 9 + 8 / 5)) < 1e-12
    assert abs(Se.sum() - h ** 3) < 1e-13


def test_free_electron_eigenvalues_converge_at_sixth_order():
    """Lowest eigenvalues of the empty lattice (V = 0) at a general k against
    |k + G|^2 / 2: the error falls by about 2^6 from a 2^3 to a 4^3 mesh, and
    the serendipity elements beat the triquadratic ones on the same mesh."""
    L = (3.0, 3.3, 2.7)
    kap = np.array([0.1, -0.23, 0.37])
    G = np.array(list(itertools.product(range(-3, 4), repeat=3)), float)
    exact = np.sort(0.5 * (((G + kap) * (2 * np.pi / np.array(L))) ** 2).sum(1))[:8]
    err = {}
    for p, m in ((3, 2), (3, 4), (2, 2)):
        o = oracle.Oracle(bare(L, (m, m, m), p=p, n=5))
        H, S = o.assemble_dense(np.zeros(o.n_qp), kap)
        ev = oracle.generalized_eigh(H, S, 8)
        err[(p, m)] = np.abs(ev - exact).max() / exact.max()
    assert err[(3, 4)] < 1e-3
    assert err[(3, 2)] / err[(3, 4)] > 25, err
    assert err[(3, 2)] < err[(2, 2)], err
