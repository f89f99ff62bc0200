"""Pins of the oracle's Bloch-periodic enrichment (eq. Psi with
f(R) = exp(i k.R); the PU functions are then periodic and the classical FE
functions keep their boundary phases):

- Psi^k(x + a_d) = exp(2 pi i kappa_d) Psi^k(x), value and gradient, with
  many overlapping images (analytic and tabulated radials), and Psi^k = Psi
  at Gamma;
- the global matrices against a direct evaluation of the global basis
  functions at the rule's points (periodic trilinear hats written out in
  numpy, with and without the boundary phase), for FE-FE, FE-enriched and
  enriched-enriched entries across the cell boundary, where images overlap;
- at Gamma (and at integer kappa) the matrices equal those of the periodic
  enrichment; H and S are Hermitian, S is positive definite, and
  H(-kappa) = conj(H(kappa));
- zone folding: the eigenvalues of a cell tripled along a_1 at Gamma are the
  union of the primitive cell's at kappa_1 = 0, 1/3, 2/3 (a geometry where no
  PU support sees two images of one atom);
- the separable term's projector coefficients over this basis against the
  global basis functions and the projectors' Bloch sums written out."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import workloads as W

KAP = (0.31, -0.17, 0.23)


def overlapping(fe_order=1, tab=False):
    """One atom in a small cell whose enrichment cutoff (3.0) exceeds half
    the cell side (4.6), so several images reach every point."""
    prob = W.small("one", mesh=(3, 3, 2), fe_order=fe_order, levels=1, n=3, a=4.6, rc=3.0, re=2.4)
    if tab:
        prob = W.with_tabulated_radials(prob, 40)
    return W.with_bloch_enrichment(prob)


@pytest.mark.parametrize("tab", [False, True])
def test_enrichment_is_bloch_periodic(tab):
    prob = overlapping(tab=tab)
    o = oracle.Oracle(prob)
    lat = np.array(prob["lattice"])
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(6):
        x = rng.uniform(0.0, 1.0, 3) @ lat
        for desc, l in ((0, 0), (1, 1)):
            for m in range(-l, l + 1):
                v0, g0 = o.enrichment_bloch(0, desc, m, x, KAP)
                assert abs(v0) > 0.0 or np.abs(g0).max() > 0.0
                for d in range(3):
                    ph = np.exp(2j * np.pi * KAP[d])
                    v1, g1 = o.enrichment_bloch(0, desc, m, x + lat[d], KAP)
                    worst = max(worst, abs(v1 - ph * v0), np.abs(g1 - ph * g0).max())
                # Gamma: the periodic enrichment
                vg, gg = o.enrichment_bloch(0, desc, m, x, (0.0, 0.0, 0.0))
                vp, gp, _ = o.enrichment(0, desc, m, x)
                assert abs(vg - vp) < 1e-15 and np.abs(gg - gp).max() < 1e-15
                assert abs(vg.imag) == 0.0
    assert worst < 1e-13


def _hats(u, j, n):
    """Trilinear hat of grid vertex j at reduced points u (any lattice shift
    T of the hat's centre is the caller's): value and reduced gradient."""
    t = u - np.asarray(j, float) / np.asarray(n, float)
    f = np.maximum(0.0, 1.0 - np.abs(t) * n)
    df = np.where(np.abs(t) * n < 1.0, -np.sign(t) * n, 0.0)
    val = f[:, 0] * f[:, 1] * f[:, 2]
    g = np.stack([df[:, 0] * f[:, 1] * f[:, 2], f[:, 0] * df[:, 1] * f[:, 2], f[:, 0] * f[:, 1] * df[:, 2]], 1)
    return val, g


def _global_hat(u, j, n, kap, inv):
    """sum_T exp(2 pi i kap.T) hat(u - T) and its Cartesian gradient."""
    val = np.zeros(len(u), complex)
    gu = np.zeros((len(u), 3), complex)
    for T in np.ndindex(3, 3, 3):
        T = np.array(T) - 1
        v, g = _hats(u - T, j, n)
        ph = np.exp(2j * np.pi * np.dot(kap, T))
        val += ph * v
        gu += ph * g
    return val, gu @ inv.T   # d/dx_c = sum_d inv[c][d] d/du_d


def test_matrices_against_global_functions():
    prob = overlapping()
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    lat = np.array(prob["lattice"])
    inv = np.linalg.inv(lat)
    n = np.array(prob["mesh"])
    u = xyz @ inv
    off = o.dof_offset()
    # global functions: the FE hats of three vertices (one inside, two on
    # the boundary layer), and every enriched function of two vertices
    funcs = {}
    for v in (0, 4, int(n[0] * n[1] * n[2]) - 1):
        j = (v % n[0], (v // n[0]) % n[1], v // (n[0] * n[1]))
        funcs[int(off[v])] = _global_hat(u, j, n, np.array(KAP), inv)
    enr_vertices = [v for v in range(len(off) - 1) if off[v + 1] - off[v] > 1][:2]
    assert len(enr_vertices) == 2
    for v in enr_vertices:
        j = (v % n[0], (v // n[0]) % n[1], v // (n[0] * n[1]))
        M, gM = _global_hat(u, j, n, np.zeros(3), inv)
        for s, (atom, desc, m) in enumerate(o.vertex_functions(v)):
            psi = np.zeros(len(u), complex)
            gpsi = np.zeros((len(u), 3), complex)
            for q in range(len(u)):
                psi[q], gpsi[q] = o.enrichment_bloch(int(atom), int(desc), int(m), xyz[q], KAP)
            funcs[int(off[v]) + 1 + s] = (M * psi, gM * psi[:, None] + M[:, None] * gpsi)
    D = sorted(funcs)
    Hd, Sd = o.assemble_dense_bloch(V, KAP)
    Hb = np.zeros((len(D), len(D)), complex)
    Sb = np.zeros_like(Hb)
    for a, i in enumerate(D):
        fi, gi = funcs[i]
        for b, jj in enumerate(D):
            fj, gj = funcs[jj]
            Sb[a, b] = np.sum(w * np.conj(fi) * fj)
            Hb[a, b] = np.sum(w * (0.5 * np.sum(np.conj(gi) * gj, 1) + V * np.conj(fi) * fj))
    Hs, Ss = Hd[np.ix_(D, D)], Sd[np.ix_(D, D)]
    assert np.abs(Ss).max() > 0 and np.abs(Hs[np.abs(Hs) > 0]).size > len(D)
    assert np.abs(Sb - Ss).max() < 1e-12 * np.abs(Ss).max()
    assert np.abs(Hb - Hs).max() < 1e-12 * np.abs(Hs).max()


@pytest.mark.parametrize("fe_order", [1, 2, 3])
def test_gamma_symmetries_and_time_reversal(fe_order):
    prob = overlapping(fe_order)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    Hp, Sp = o.assemble_dense(V, (0.0, 0.0, 0.0))
    for kap in ((0.0, 0.0, 0.0), (1.0, 0.0, -1.0)):
        Hg, Sg = o.assemble_dense_bloch(V, kap)
        assert np.abs(Hg - Hp).max() < 1e-12 * np.abs(Hp).max()
        assert np.abs(Sg - Sp).max() < 1e-12 * np.abs(Sp).max()
    H, S = o.assemble_dense_bloch(V, KAP)
    assert np.abs(H - H.conj().T).max() == 0.0 and np.abs(S - S.conj().T).max() == 0.0
    assert np.linalg.eigvalsh(S).min() > 0.0
    Hm, Sm = o.assemble_dense_bloch(V, tuple(-k for k in KAP))
    assert np.abs(Hm - H.conj()).max() < 1e-13 * np.abs(H).max()
    assert np.abs(Sm - S.conj()).max() < 1e-13 * np.abs(S).max()
    # not the periodic form's matrices away from Gamma
    Ha, _ = o.assemble_dense(V, KAP)
    assert np.abs(np.linalg.eigvalsh(H) - np.linalg.eigvalsh(Ha)).max() > 1e-6


def folding_pair(fe_order):
    """A cell long along a_1 (6 x 3.2 x 3.2, one atom, s and p functions,
    rc = 2.0, re = 1.0) and the same crystal in a cell tripled along a_1.
    The nearest other image along a_1 is 6 bohr away, farther than
    re + (PU support diagonal 2.7) + rc, so a PU support never sees two images
    of the atom and the tripled cell's basis splits into the primitive
    cell's Bloch bases at kappa_1 = 0, 1/3, 2/3."""
    tau = np.array([1.1, 1.3, 1.7])
    enr = [{"species": 0, "l": 0, "a": 1.2, "rc": 2.0, "re": 1.0},
           {"species": 0, "l": 1, "a": 0.8, "rc": 2.0, "re": 1.0}]
    info = [{"name": "X", "Z": 2.0, "rloc": 0.5}]
    quad = {"n": 3, "n_ref": 6, "levels": 1, "mode": "geom", "dist": 1.0, "tol": 1e-6}
    prim = W._problem([[6.0, 0, 0], [0, 3.2, 0], [0, 0, 3.2]], (4, 2, 2), fe_order, [tau], [0], info, enr,
                      quad, [[0, 0, 0]], 4, "fold-primitive")
    sup = W._problem([[18.0, 0, 0], [0, 3.2, 0], [0, 0, 3.2]], (12, 2, 2), fe_order,
                     [tau, tau + [6.0, 0, 0], tau + [12.0, 0, 0]], [0, 0, 0], info, enr, quad, [[0, 0, 0]], 4,
                     "fold-tripled")
    assert 6.0 - 1.0 - np.sqrt(1.5 ** 2 + 2 * 1.6 ** 2) > 2.0
    return W.with_bloch_enrichment(prim), sup


@pytest.mark.parametrize("fe_order", [1, 2])
def test_zone_folding(fe_order):
    prim, sup = folding_pair(fe_order)
    op, os_ = oracle.Oracle(prim), oracle.Oracle(sup)
    assert os_.n_dof == 3 * op.n_dof
    xp, _, _ = op.quadrature()
    xs, _, _ = os_.quadrature()
    Vp, Vs = oracle.potential_np(xp, prim), oracle.potential_np(xs, sup)
    Hs, Ss = os_.assemble_dense(Vs, (0.0, 0.0, 0.0))
    es = sl.eigh(Hs, Ss, eigvals_only=True)
    ep = []
    for k1 in (0.0, 1.0 / 3.0, 2.0 / 3.0):
        H, S = op.assemble_dense_bloch(Vp, (k1, 0.0, 0.0))
        ep.append(sl.eigh(H, S, eigvals_only=True))
    ep = np.sort(np.concatenate(ep))
    m = 40
    assert np.abs(ep[:m] - es[:m]).max() < 1e-8 * max(1.0, np.abs(es[:m]).max())


def test_nonlocal_coefficients_against_global_functions():
    """Projector coefficients of the separable term over the Bloch-periodic
    basis: f_J^i = sum_q w_q conj(Phi_i(x_q)) P_J(x_q) with the global basis
    functions written out as in test_matrices_against_global_functions and the
    projector's Bloch sum P_J = sum_n exp(2 pi i kappa.n) v_J(x - tau - n.a),
    v = exp(-a r^2)(1 - r^2/rc^2)^3 S_lm (the synthetic projector); the FE
    rows equal those of the periodic form's coefficients."""
    prob = W.with_projectors(overlapping())
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    lat = np.array(prob["lattice"])
    inv = np.linalg.inv(lat)
    n = np.array(prob["mesh"])
    u = xyz @ inv
    off = o.dof_offset()
    Fb = o.nonlocal_f(KAP, bloch=True)
    Fp = o.nonlocal_f(KAP)
    fe = np.concatenate([np.arange(off[v], off[v] + 1) for v in range(o.n_vertex)])
    assert np.abs(Fb[:, fe] - Fp[:, fe]).max() == 0.0
    # projector functions J in the oracle's order: descriptor, atom, m
    tau = np.array(prob["atoms"][0])
    Pj = []
    for q in prob["projectors"]:
        for m in range(-q["l"], q["l"] + 1):
            val = np.zeros(len(u), complex)
            for img in np.ndindex(5, 5, 5):
                nn = np.array(img) - 2
                r = xyz - tau - nn @ lat
                sq = np.sum(r * r, 1)
                inside = sq < q["rc"] ** 2
                S = np.array([oracle.solid_harmonic(q["l"], m, rr)[0] if ok else 0.0 for rr, ok in zip(r, inside)])
                v = np.where(inside, np.exp(-q["a"] * sq) * np.clip(1 - sq / q["rc"] ** 2, 0, None) ** 3 * S, 0.0)
                val += np.exp(2j * np.pi * np.dot(KAP, nn)) * v
            Pj.append(val)
    v = [v for v in range(len(off) - 1) if off[v + 1] - off[v] > 1][0]
    j = (v % n[0], (v // n[0]) % n[1], v // (n[0] * n[1]))
    M, _ = _global_hat(u, j, n, np.zeros(3), inv)
    for s, (atom, desc, m) in enumerate(o.vertex_functions(v)):
        psi = np.array([o.enrichment_bloch(int(atom), int(desc), int(m), x, KAP)[0] for x in xyz])
        phi = M * psi
        for J, P in enumerate(Pj):
            want = np.sum(w * np.conj(phi) * P)
            assert abs(Fb[J, off[v] + 1 + s] - want) < 1e-12 * max(1.0, abs(want))
