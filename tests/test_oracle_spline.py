"""Pins of the oracle's tabulated radial functions (section "Partition of
unity enrichment functions"): the radial is r^l times the cubic spline fit of
the sampled pseudoatomic radial (over r^l) times the C^3 cutoff
h(r, rc) = 1 + 20 x^7 - 70 x^6 + 84 x^5 - 35 x^4, x = r/rc.

Each test checks a closed form or an exact property: a cubic is reproduced
exactly by the clamped spline, the spline error falls as the fourth power of
the knot spacing, h(0) = 1 and the clamped slope at the nucleus, the
function and its gradient vanish at rc, the first radial moment of h is
rc^3/18, and derivatives agree with finite differences."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def h_paper(r, rc):
    x = np.minimum(np.asarray(r, float) / rc, 1.0)
    return 1 + 20 * x ** 7 - 70 * x ** 6 + 84 * x ** 5 - 35 * x ** 4


def one_atom(l, rc, samples, L=7.0, tau=(3.1, 3.4, 2.9), mesh=2, n=3, levels=0, re=1.0):
    prob = {
        "lattice": [[L, 0, 0], [0, L, 0], [0, 0, L]], "mesh": [mesh] * 3, "fe_order": 1,
        "atoms": [list(tau)], "species": [0], "species_info": [{"name": "X", "Z": 1.0, "rloc": 0.5}],
        "enrichments": [{"species": 0, "l": l, "a": 1.0, "rc": rc, "re": re, "radial": list(samples)}],
        "quad": {"n": n, "n_ref": n + 3, "levels": levels, "mode": "geom", "dist": 2.5, "tol": 1e-6},
        "kpts": [[0, 0, 0]], "n_eig": 4, "potential": {"cutoff": 12.0},
    }
    return prob


def points_in_ball(tau, rc, k, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rng.uniform(0.02, 0.98, size=k) * rc
    return np.asarray(tau) + d * r[:, None], r


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_clamped_spline_reproduces_a_cubic(l):
    """Samples t_j = p(r_j)/h(r_j) with p(r) = 1 - 3x^2 + 2x^3 (zero slope at
    0 and at rc, p(rc) = 0) make the spline data a cubic with the clamped end
    slopes, which the spline reproduces exactly: Psi~ = p(r) S_lm."""
    rc, n = 2.4, 13
    r = np.linspace(0, rc, n)
    x = r / rc
    p = 1 - 3 * x * x + 2 * x ** 3
    t = np.zeros(n)
    t[:-1] = p[:-1] / h_paper(r[:-1], rc)
    prob = one_atom(l, rc, t)
    o = oracle.Oracle(prob)
    tau = np.asarray(prob["atoms"][0])
    xs, rr = points_in_ball(tau, rc, 20, seed=l)
    for xq, rq in zip(xs, rr):
        xx = rq / rc
        pv = 1 - 3 * xx * xx + 2 * xx ** 3
        dp = (-6 * xx + 6 * xx * xx) / rc
        for m in range(-l, l + 1):
            v, g, _ = o.enrichment(0, 0, m, xq)
            S, dS, _ = oracle.solid_harmonic(l, m, xq - tau)
            rhat = (xq - tau) / rq
            assert abs(v - pv * S) < 1e-13 * max(1.0, abs(S))
            assert np.abs(g - (dp * rhat * S + pv * dS)).max() < 1e-12 * max(1.0, np.abs(dS).max())


def test_spline_error_falls_as_fourth_power_of_spacing():
    """Samples of exp(-a r^2): the spline of exp(-a r^2) h(r) converges to it
    at fourth order in the knot spacing (errors at fixed off-knot radii)."""
    rc, a = 2.6, 1.1
    rq = np.linspace(0.013, 0.987, 57) * rc
    errs = []
    for n in (17, 33, 65):
        r = np.linspace(0, rc, n)
        prob = one_atom(0, rc, np.exp(-a * r * r))
        o = oracle.Oracle(prob)
        tau = np.asarray(prob["atoms"][0])
        y00 = 0.5 / math.sqrt(math.pi)
        e = 0.0
        for x in rq:
            v, _, _ = o.enrichment(0, 0, 0, tau + np.array([x, 0, 0]))
            e = max(e, abs(v / y00 - math.exp(-a * x * x) * h_paper(x, rc)))
        errs.append(e)
    assert errs[-1] < 2e-6
    for e0, e1 in zip(errs, errs[1:]):
        assert 10.0 < e0 / e1 < 24.0, errs


def test_nucleus_and_cutoff():
    """At the nucleus the s function equals t_0 Y_00 (h(0) = 1) with zero
    gradient (clamped slope); toward rc the value falls like (rc - r)^2 and
    the gradient like (rc - r), and both are zero beyond rc."""
    rc, n = 2.2, 23
    r = np.linspace(0, rc, n)
    t = 0.7 * np.exp(-0.9 * r * r)
    prob = one_atom(0, rc, t)
    o = oracle.Oracle(prob)
    tau = np.asarray(prob["atoms"][0])
    y00 = 0.5 / math.sqrt(math.pi)
    v, g, hs = o.enrichment(0, 0, 0, tau)
    assert abs(v - 0.7 * y00) < 1e-15 and np.abs(g).max() == 0.0
    assert np.all(np.isfinite(hs))
    d = np.array([0.48, -0.6, 0.64])
    vals, grads = [], []
    for eps in (1e-2, 5e-3):
        v, g, _ = o.enrichment(0, 0, 0, tau + (rc - eps) * d)
        vals.append(abs(v))
        grads.append(np.linalg.norm(g))
    assert 3.0 < vals[0] / vals[1] < 5.0 and 1.5 < grads[0] / grads[1] < 2.5
    v, g, hs = o.enrichment(0, 0, 0, tau + (rc + 1e-9) * d)
    assert v == 0.0 and np.abs(g).max() == 0.0 and np.abs(hs).max() == 0.0


def test_cutoff_moment_through_the_partition_of_unity():
    """With constant samples the s function is spline(h) Y_00, whose integral
    tends to 4 pi Y_00 rc^3/18 = sqrt(pi) rc^3 / 9 (the first radial moment
    of h is rc^3/18).  Every vertex carries the function and the FE functions
    sum to one, so the integral is 1_FE^T S 1_enr."""
    rc, n = 2.3, 65
    prob = one_atom(0, rc, np.ones(n), L=6.0, tau=(2.3, 2.9, 3.4), n=10, levels=2, re=100.0)
    o = oracle.Oracle(prob)
    _, S = o.assemble_dense(np.zeros(o.n_qp))
    off = o.dof_offset()
    fe = np.zeros(o.n_dof)
    enr = np.zeros(o.n_dof)
    for v in range(o.n_vertex):
        fe[off[v]] = 1.0
        enr[off[v] + 1] = 1.0
    exact = math.sqrt(math.pi) * rc ** 3 / 9.0
    got = fe @ S.real @ enr
    assert abs(got - exact) < 2e-6 * exact, (got, exact)


def test_tabulated_enrichment_periodic_and_derivatives():
    """Gradients and Hessians of the periodic tabulated enrichment functions
    (l = 0 .. 3, several images) agree with central differences, and the
    functions are lattice periodic."""
    prob = W.with_tabulated_radials(W.small("ceal", mesh=(2, 2, 2), fe_order=1, levels=0, n=2, a=4.0, rc=2.6),
                                    n_samples=40)
    o = oracle.Oracle(prob)
    lat = np.asarray(prob["lattice"])
    rng = np.random.default_rng(5)
    for desc in range(len(prob["enrichments"])):
        l = prob["enrichments"][desc]["l"]
        atom = prob["enrichments"][desc]["species"]
        for _ in range(3):
            x = rng.uniform(0, 4.0, size=3)
            m = int(rng.integers(-l, l + 1))
            v, g, h = o.enrichment(atom, desc, m, x)
            v2, g2, _ = o.enrichment(atom, desc, m, x + lat[0] - lat[2])
            assert abs(v - v2) < 1e-13 and np.abs(g - g2).max() < 1e-12
            eps = 1e-5
            for k in range(3):
                dx = np.zeros(3)
                dx[k] = eps
                vp, gp, _ = o.enrichment(atom, desc, m, x + dx)
                vm, gm, _ = o.enrichment(atom, desc, m, x - dx)
                assert abs((vp - vm) / (2 * eps) - g[k]) < 1e-7 * max(1, abs(g).max())
                assert np.abs((gp - gm) / (2 * eps) - h[:, k]).max() < 1e-6 * max(1, np.abs(h).max())
