"""Pins of the oracle's separable nonlocal term (eq. disceig3d):

    Vnl_ij = sum_J h_J f_J^i conj(f_J^j),
    f_J^i  = int phi_i^* sum_n exp(i k . a_n) v_J(x - tau - a_n) dx,

with synthetic projectors v = exp(-a r^2) (1 - r^2/rc^2)^3 r^l Y_lm.  Each pin
checks something the definition fixes without restating it: the partition of
unity of the classical FE functions (their f summed is the projector's
integral over all space, a 1D radial closed form, also when the projector's
support crosses the cell boundary and its images matter), Hermitian
positive semi-definiteness with rank equal to the number of projector
functions, Bloch periodicity and time reversal in k, invariance under a
lattice translation of the atom, convergence with the quadrature rule, and
the min-max consequence for eigenvalues (a positive separable term can only
raise each Ritz value).
"""
import numpy as np
import pytest

import oracle
from test_oracle_pins import bare, diag


def _radial_int_l0(a, rc):
    x, w = np.polynomial.legendre.leggauss(200)
    r = 0.5 * rc * (x + 1)
    w = 0.5 * rc * w
    Y00 = 0.5 / np.sqrt(np.pi)
    return 4 * np.pi * Y00 * np.sum(w * r * r * np.exp(-a * r * r) * (1 - (r / rc) ** 2) ** 3)


def _prob(atom, levels=2, n=6, enrich=False, p=1, mesh=(3, 3, 3), L=5.0, projectors=None, dist=0.6):
    enr = [{"species": 0, "l": 0, "a": 1.1, "rc": 2.0, "re": 1.5}] if enrich else []
    pr = bare(diag(L, L, L), mesh, p, n=n, enrichments=enr, atoms=(atom,), levels=levels)
    pr["quad"]["dist"] = dist
    pr["projectors"] = projectors or [{"species": 0, "l": 0, "a": 1.5, "rc": 1.8, "h": 0.7},
                                      {"species": 0, "l": 1, "a": 2.0, "rc": 1.6, "h": -0.4}]
    return pr


@pytest.mark.parametrize("atom,enrich", [((2.3, 2.6, 2.1), False), ((0.2, 4.9, 0.3), False),
                                          ((0.2, 4.9, 0.3), True)])
def test_fe_partition_of_unity_gives_projector_integral(atom, enrich):
    """Gamma point: the classical FE functions sum to 1, so summing f_J^i over
    the FE DOFs gives the integral of the projector over all space: the radial
    closed form for l = 0, zero for l = 1 (the atom near a corner: its images
    across the cell faces carry the rest of the support).  The rule refines
    two levels over the whole projector support (8^3 points per leaf), which
    integrates it to about 2e-10."""
    pr = _prob(atom, enrich=enrich, levels=2, n=8, dist=2.0)
    o = oracle.Oracle(pr)
    F = o.nonlocal_f((0.0, 0.0, 0.0))
    assert F.shape[0] == 1 + 3
    off = o.dof_offset()
    fe = np.array([off[v] for v in range(o.n_vertex)])   # trilinear: one FE slot per vertex, first
    I0 = _radial_int_l0(1.5, 1.8)
    assert abs(F[0, fe].sum() - I0) < 2e-9 * I0
    assert np.abs(F[0, fe].imag).max() == 0.0
    for J in (1, 2, 3):
        assert abs(F[J, fe].sum()) < 2e-9 * I0


def test_hermitian_psd_rank_and_sign():
    pr = _prob((1.1, 2.6, 3.9), enrich=True, p=2, mesh=(2, 3, 2), levels=1, n=4)
    o = oracle.Oracle(pr)
    kap = (0.12, -0.24, 0.37)
    pos = [dict(q, h=abs(q["h"])) for q in pr["projectors"]]
    Vn = o.nonlocal_dense(kap, pos)
    assert np.array_equal(Vn, Vn.conj().T)
    ev = np.linalg.eigvalsh(Vn)
    scale = np.abs(ev).max()
    assert ev.min() > -1e-13 * scale
    assert int((ev > 1e-10 * scale).sum()) == 4     # one s and three p projector functions
    neg = o.nonlocal_dense(kap, [dict(q, h=-abs(q["h"])) for q in pr["projectors"]])
    np.testing.assert_allclose(neg, -Vn, rtol=0, atol=1e-15 * scale)


def test_bloch_periodicity_time_reversal_and_translation():
    pr = _prob((1.1, 2.6, 3.9), enrich=True, p=2, mesh=(2, 3, 2), levels=1, n=4)
    o = oracle.Oracle(pr)
    kap = np.array([0.12, -0.24, 0.37])
    V0 = o.nonlocal_dense(kap)
    scale = np.abs(V0).max()
    assert np.abs(o.nonlocal_dense(kap + np.array([1.0, -2.0, 1.0])) - V0).max() < 1e-13 * scale
    assert np.abs(o.nonlocal_dense(-kap) - V0.conj()).max() < 1e-13 * scale
    # the atom moved by a lattice vector: the same projector images
    pr2 = dict(pr, atoms=[[1.1 + 5.0, 2.6, 3.9 - 5.0]])
    o2 = oracle.Oracle(pr2)
    assert o2.n_dof == o.n_dof
    assert np.abs(o2.nonlocal_dense(kap) - V0).max() < 1e-12 * scale


def test_converges_with_the_rule():
    """f on a fixed basis converges as the rule over the projector support is
    refined (against a fine rule: two levels, 8^3 points per leaf)."""
    errs = []
    ref = None
    for levels, n in ((2, 8), (0, 3), (1, 4), (2, 5)):
        pr = _prob((2.3, 2.6, 2.1), levels=levels, n=n, dist=2.0)
        F = oracle.Oracle(pr).nonlocal_f((0.1, 0.2, -0.3))
        if ref is None:
            ref = F
        else:
            errs.append(np.abs(F - ref).max() / np.abs(ref).max())
    assert errs[0] > 100 * errs[1] > 1e4 * errs[2]
    assert errs[2] < 1e-7


def test_positive_term_raises_every_ritz_value():
    pr = _prob((1.1, 2.6, 3.9), enrich=True, p=2, mesh=(2, 3, 2), levels=1, n=4)
    o = oracle.Oracle(pr)
    kap = (0.12, -0.24, 0.37)
    xyz, _, _ = o.quadrature()
    H, S = o.assemble_dense(oracle.potential_np(xyz, pr), kap)
    Vn = o.nonlocal_dense(kap, [dict(q, h=abs(q["h"])) for q in pr["projectors"]])
    e0 = oracle.generalized_eigh(H, S, 12)
    e1 = oracle.generalized_eigh(H + Vn, S, 12)
    assert np.all(e1 >= e0 - 1e-10)
    assert (e1 - e0).max() > 1e-3
