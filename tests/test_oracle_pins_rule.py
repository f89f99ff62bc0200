"""Two-sided pins of the oracle's quadrature rules and checks of its sampled
(block / per-element) functions against its dense ones.

The geometric rule is checked against an exact point-to-box distance written
here (the closest point of a box to a point is the point clamped into the
box, taken over the 27 nearest lattice images in 3D at once), in both
directions: a split cell lies within the refinement distance and an unsplit
leaf below the maximum level lies beyond it.  The error-driven rule of
section "Adaptive quadrature" is checked the same way with the base and
reference Gauss rules of numpy, for both of the paper's integrands, Psi^2
and |grad Psi|^2.  The refined-element and point counts of the two
benchmark cells were computed independently of the oracle (from the same
criterion with a clamp over image shells) when the workloads were specified.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W

from test_oracle_pins import _radial_integrals, bare, diag


def _box(prob, e, lev, c):
    """Cartesian box [lo, hi] of octree cell (lev, c) of element e of an
    orthorhombic cell."""
    mesh = np.asarray(prob["mesh"])
    L = np.diag(np.asarray(prob["lattice"], float))
    i = np.array([e % mesh[0], (e // mesh[0]) % mesh[1], e // (mesh[0] * mesh[1])])
    h = L / mesh
    s = 1.0 / 2 ** lev
    lo = (i + np.asarray(c) * s) * h
    return lo, lo + s * h


def _box_nucleus_distance(prob, lo, hi):
    """Exact distance from the box to the nearest nucleus image: clamp every
    image into the box and take the shortest gap."""
    L = np.diag(np.asarray(prob["lattice"], float))
    atoms = np.asarray(prob["atoms"], float)
    shifts = np.array(list(itertools.product((-1, 0, 1), repeat=3)), float) * L
    best = np.inf
    for A in atoms:
        # the image nearest the box centre, then its 27 neighbours
        ctr = 0.5 * (lo + hi)
        base = A - L * np.round((A - ctr) / L)
        imgs = base + shifts
        gap = imgs - np.clip(imgs, lo, hi)
        best = min(best, np.sqrt((gap * gap).sum(1)).min())
    return best


def _tree(lev, ijk, loff, e):
    """Internal (split) cells of element e's octree: every ancestor of a leaf."""
    internal = set()
    for k in range(loff[e], loff[e + 1]):
        l, c = int(lev[k]), ijk[k].astype(int)
        for up in range(1, l + 1):
            internal.add((l - up, tuple(int(x) for x in (c >> up))))
    return internal


def _check_geom_rule(prob, elems=None):
    o = oracle.Oracle(prob)
    lev, ijk, loff = o.leaves()
    d, Lmax = prob["quad"]["dist"], prob["quad"]["levels"]
    n_split = n_leaf = 0
    for e in (range(o.n_elem) if elems is None else elems):
        for (l, c) in _tree(lev, ijk, loff, e):
            assert l < Lmax
            assert _box_nucleus_distance(prob, *_box(prob, e, l, c)) <= d + 1e-12
            n_split += 1
        for k in range(loff[e], loff[e + 1]):
            if lev[k] < Lmax:
                assert _box_nucleus_distance(prob, *_box(prob, e, lev[k], ijk[k])) > d - 1e-12
                n_leaf += 1
    return n_split, n_leaf


@pytest.mark.parametrize("levels,dist", [(2, 1.0), (3, 0.7)])
def test_geometric_rule_two_sided_small(levels, dist):
    """Every split cell lies within dist of a nucleus image and every unsplit
    leaf below the maximum level lies beyond it (exact box distances)."""
    prob = W.small("lih", mesh=(3, 2, 3), fe_order=2, levels=levels, n=3, a=5.0)
    prob["quad"]["dist"] = dist
    n_split, n_leaf = _check_geom_rule(prob)
    assert n_split > 0 and n_leaf > 0


def _refined_sample(prob, o, count, seed):
    """Some refined elements and some of their unrefined neighbours."""
    _, _, loff = o.leaves()
    nl = np.diff(loff)
    rng = np.random.default_rng(seed)
    ref = np.nonzero(nl > 1)[0]
    plain = np.nonzero(nl == 1)[0]
    return list(rng.choice(ref, size=min(count, ref.size), replace=False)) + \
        list(rng.choice(plain, size=min(count, plain.size), replace=False))


@pytest.mark.parametrize("name,n_ref,n_qp", [("lih_cell", 231, 1519776), ("ceal_cell", 176, 27262976)])
def test_benchmark_cells_rule_counts_and_sample(name, n_ref, n_qp):
    """Refined-element and point counts of the two benchmark cells (computed
    independently of the oracle when the workloads were specified), and the
    two-sided rule check on a seeded sample of their elements."""
    prob = getattr(W, name)()
    o = oracle.Oracle(prob)
    _, _, loff = o.leaves()
    assert int((np.diff(loff) > 1).sum()) == n_ref
    assert o.n_qp == n_qp
    _check_geom_rule(prob, _refined_sample(prob, o, 6, seed=11))


# ------------------------------------------------------------- error mode

def _element_functions(o, prob, e):
    mesh = prob["mesh"]
    i = (e % mesh[0], (e // mesh[0]) % mesh[1], e // (mesh[0] * mesh[1]))
    fns = set()
    for c in range(8):
        j = [(i[d] + ((c >> d) & 1)) % mesh[d] for d in range(3)]
        v = (j[2] * mesh[1] + j[1]) * mesh[0] + j[0]
        for f in o.vertex_functions(v):
            fns.add(tuple(int(x) for x in f))
    return sorted(fns)


def _cell_errors(o, prob, e, lev, c, fn, n, nref):
    """|Q_n - Q_ref| of Psi^2 and of |grad Psi|^2 on the cell, tensor Gauss
    rules from numpy, the map of the element written out here."""
    mesh = np.asarray(prob["mesh"])
    lat = np.asarray(prob["lattice"], float)
    i = np.array([e % mesh[0], (e // mesh[0]) % mesh[1], e // (mesh[0] * mesh[1])])
    vol = abs(np.linalg.det(lat)) / mesh.prod()
    out = []
    for m in (n, nref):
        x, w = np.polynomial.legendre.leggauss(m)
        s = 1.0 / 2 ** lev
        t = (np.asarray(c)[:, None] + 0.5 * (x[None, :] + 1.0)) * s   # in [0, 1] per direction
        I0 = I1 = 0.0
        for a3 in range(m):
            for a2 in range(m):
                for a1 in range(m):
                    red = (i + np.array([t[0, a1], t[1, a2], t[2, a3]])) / mesh
                    X = red @ lat
                    wt = w[a1] * w[a2] * w[a3] * (0.5 * s) ** 3 * vol
                    v, g, _ = o.enrichment(fn[0], fn[1], fn[2], X)
                    I0 += wt * v * v
                    I1 += wt * g @ g
        out.append((I0, I1))
    return abs(out[0][0] - out[1][0]), abs(out[0][1] - out[1][1])


def test_error_driven_rule_two_sided_and_gradient_criterion():
    """The error-driven rule: a cell is split iff one of the functions still
    tested on it misses the tolerance for Psi^2 or |grad Psi|^2 (only those
    are tested on its children); unsplit leaves below the maximum level meet
    it for every tested function.  With an l = 1 function the gradient
    integrand is the binding one on some cells.  The rule then integrates
    |grad Psi|^2 of the isolated function to its radial closed form."""
    enr = [{"species": 0, "l": 1, "a": 2.5, "rc": 1.8, "re": 1.6}]
    prob = bare(diag(4.0, 4.0, 4.0), (2, 2, 2), 1, n=3, enrichments=enr, atoms=((1.3, 2.2, 1.9),))
    prob["quad"] = {"n": 3, "n_ref": 6, "levels": 3, "mode": "error", "dist": 0, "tol": 1e-6}
    tol, Lmax = 1e-6, 3
    o = oracle.Oracle(prob)
    lev, ijk, loff = o.leaves()
    assert lev.max() >= 2
    grad_only = 0
    for e in range(o.n_elem):
        internal = _tree(lev, ijk, loff, e)
        tested = {(0, (0, 0, 0)): _element_functions(o, prob, e)}
        # walk the internal cells top down: the failing functions pass on
        for l in range(Lmax + 1):
            for cell in sorted(x for x in internal if x[0] == l):
                fns = tested[cell]
                fails = []
                for fn in fns:
                    e0, e1 = _cell_errors(o, prob, e, l, cell[1], fn, 3, 6)
                    if e0 > tol or e1 > tol:
                        fails.append(fn)
                        grad_only += int(e1 > tol and e0 <= tol)
                assert fails, (e, cell)
                for ch in range(8):
                    cc = tuple(2 * cell[1][d] + ((ch >> d) & 1) for d in range(3))
                    tested[(l + 1, cc)] = fails
        for k in range(loff[e], loff[e + 1]):
            key = (int(lev[k]), tuple(int(x) for x in ijk[k]))
            if key[0] < Lmax:
                for fn in tested.get(key, []):
                    e0, e1 = _cell_errors(o, prob, e, key[0], key[1], fn, 3, 6)
                    assert e0 <= tol and e1 <= tol, (e, key, fn, e0, e1)
    assert grad_only > 0
    xyz, w, _ = o.quadrature()
    _, I1 = _radial_integrals(1, 2.5, 1.8)
    for m in (-1, 0, 1):
        got = sum(wq * (lambda g: g @ g)(o.enrichment(0, 0, m, xq)[1]) for xq, wq in zip(xyz, w))
        assert abs(got - I1) < 1e-6 * len(lev)


# ------------------------------------------- sampled functions vs dense ones

def test_assemble_block_equals_dense_blocks():
    """or_assemble_block, the checker of the full-size GPU tests, gives every
    vertex block of the dense assembly (zero blocks included) at a
    non-Gamma k-point."""
    prob = W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0)
    kap = (0.12, -0.24, 0.37)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    H, S = o.assemble_dense(V, kap)
    off = o.dof_offset()
    for v in range(o.n_vertex):
        for w in range(o.n_vertex):
            Hb, Sb = o.assemble_block(V, kap, v, w)
            np.testing.assert_array_equal(Hb, H[off[v]:off[v + 1], off[w]:off[w + 1]])
            np.testing.assert_array_equal(Sb, S[off[v]:off[v + 1], off[w]:off[w + 1]])


def test_backward_element_sums_to_dense_adjoint():
    """or_backward_element, summed over the elements, gives or_backward_dense
    (dL/dV element by element, dL/dR summed) at a non-Gamma k-point."""
    prob = W.small("lih", mesh=(2, 2, 3), fe_order=2, levels=1, n=3, a=4.6, re=1.6, rc=2.0)
    kap = np.array([0.12, -0.24, 0.37])
    o = oracle.Oracle(prob)
    xyz, _, qoff = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    C = W.adjoint_factor(o.n_dof, rank=5, seed=2)
    P = C @ C.conj().T
    Cq = W.adjoint_factor(o.n_dof, rank=3, seed=3)
    Q = Cq @ Cq.conj().T
    dV, dR = o.backward_dense(V, kap, P, Q)
    dR_sum = np.zeros_like(dR)
    for e in range(o.n_elem):
        g, _ = o.element_dofs(e)
        dVe, dRe = o.backward_element(e, V[qoff[e]:qoff[e + 1]], kap, P[np.ix_(g, g)], Q[np.ix_(g, g)])
        np.testing.assert_allclose(dVe, dV[qoff[e]:qoff[e + 1]], rtol=1e-12, atol=1e-14 * np.abs(dV).max())
        dR_sum += dRe
    np.testing.assert_allclose(dR_sum, dR, rtol=1e-11, atol=1e-12 * np.abs(dR).max())
