"""GPU parity of the tabulated (spline) radial functions against the oracle,
through the C ABI (section "Partition of unity enrichment functions": the
radial is r^l times the cubic spline fit of the sampled pseudoatomic radial
times the C^3 cutoff).  The library fits its own spline from the samples; the
oracle fits its own.  Assembly (FP64 to 1e-12, bf16x6 to 1e-7), the
error-driven rule built from the tabulated functions (ties only, then
assembly on the oracle's rule), the adjoint (to 1e-11), and element matrices
of the LiH-like cell at full size with tabulated radials."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_00731_amd as P  # noqa: E402
from workloads.potential import potential_at  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_inputs(prob):
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    return o, V


CASES = {
    "lih-p2": (lambda: W.with_tabulated_radials(W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0), 40),
               [(0.0, 0.0, 0.0), (0.12, -0.24, 0.37)]),
    "one-p1-coarse": (lambda: W.with_tabulated_radials(W.small("one", mesh=(3, 3, 2), fe_order=1, levels=2, n=3,
                                                               a=4.6), 6), [(0.31, 0.0, -0.2)]),
    "ceal-l3": (lambda: W.with_tabulated_radials(W.small("ceal", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4,
                                                         rc=3.0, re=2.4), 64), [(0.0, 0.0, 0.0), (0.25, -0.25, 0.25)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_tabulated_assembly_matches_oracle(name):
    make, kpts = CASES[name]
    prob = make()
    say("tabulated assembly", name)
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    Vd = torch.from_numpy(V).cuda()
    H, S = p.assemble(Vd, kpts)
    Hs, Ss = p.assemble(Vd, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense(V, kap)
        eh = rel(p.to_dense(H[k]).cpu().numpy(), Ho)
        es = rel(p.to_dense(S[k]).cpu().numpy(), So)
        e6 = max(rel(p.to_dense(Hs[k]).cpu().numpy(), Ho), rel(p.to_dense(Ss[k]).cpu().numpy(), So))
        say(name, kap, "H", eh, "S", es, "bf16x6", e6)
        assert eh < 1e-12 and es < 1e-12 and e6 < 1e-7
    p.close()


def test_tabulated_differs_from_analytic():
    """The tabulated functions are the paper's radial (spline of the radial
    times the C^3 cutoff), not the analytic one: the two S differ by far more
    than the parity tolerance, so the tests above see the spline path."""
    base = W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)
    say("tabulated vs analytic")
    out = []
    for prob in (base, W.with_tabulated_radials(base, 40)):
        p = P.Problem(prob).setup()
        xyz, _, _ = p.quadrature()
        V = potential_at(xyz, prob)
        _, S = p.assemble(V, [(0.0, 0.0, 0.0)])
        out.append(p.to_dense(S[0]).cpu().numpy())
        p.close()
    assert rel(out[1], out[0]) > 1e-3


def test_tabulated_error_rule_and_shared_rule():
    """The error-driven rule built from tabulated functions on the GPU agrees
    with the oracle's except at ties (an error estimate within 1e-9 of the
    tolerance); on the oracle's rule H and S match to 1e-12."""
    from test_gpu_parity import RULE_TIE, _rule_cells
    from test_oracle_pins_rule import _cell_errors, _element_functions
    prob = W.with_tabulated_radials(W.small("lih", mesh=(2, 2, 3), fe_order=2, a=4.8, re=1.6, rc=2.0), 32)
    prob["quad"] = {"n": 3, "n_ref": 6, "levels": 3, "mode": "error", "dist": 0.0, "tol": 1e-6}
    q = prob["quad"]
    say("tabulated error rule")
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    glev, gijk, goff = P.pufe_get_leaves(p.ctx)
    olev, oijk, ooff = o.leaves()
    gl, gi = _rule_cells(glev, gijk, goff)
    ol, oi = _rule_cells(olev, oijk, ooff)
    decided = (gl & oi) | (ol & gi)
    for (e, l, *c) in sorted(decided):
        near = min(min(abs(x - q["tol"]) for x in _cell_errors(o, prob, e, l, c, fn, q["n"], q["n_ref"]))
                   for fn in _element_functions(o, prob, e))
        assert near <= RULE_TIE, (e, l, c, near)
    say("cells decided differently", len(decided), "leaves", len(olev))
    assert max(olev) >= 1   # the rule refines
    p.set_rule(olev, oijk, ooff)
    Vd = torch.from_numpy(V).cuda()
    kap = (0.1, -0.2, 0.3)
    H, S = p.assemble(Vd, [kap])
    Ho, So = o.assemble_dense(V, kap)
    eh, es = rel(p.to_dense(H[0]).cpu().numpy(), Ho), rel(p.to_dense(S[0]).cpu().numpy(), So)
    say("tabulated error rule H", eh, "S", es)
    assert eh < 1e-12 and es < 1e-12
    p.close()


def test_tabulated_adjoint_matches_oracle():
    """dL/dV and dL/dR (which needs the Hessians of the spline functions)
    against the oracle's dense adjoint at a general k-point."""
    from test_gpu_backward import bsr_index
    prob = W.with_tabulated_radials(W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=4.8, re=1.7,
                                            rc=2.1), 36)
    say("tabulated adjoint")
    o, V = oracle_inputs(prob)
    Cp = W.adjoint_factor(o.n_dof, rank=6, seed=0)
    Cq = W.adjoint_factor(o.n_dof, rank=3, seed=1)
    Pd, Qd = Cp @ Cp.conj().T, Cq @ Cq.conj().T
    kap = (0.12, -0.24, 0.37)
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    dV, dR = p.backward(torch.from_numpy(V).cuda(), kap, Pb, Qb)
    ev = rel(dV.cpu().numpy(), dV_o)
    er = np.abs(dR.cpu().numpy() - dR_o).max() / np.abs(dR_o).max()
    say("tabulated adjoint dL/dV", ev, "dL/dR", er)
    assert ev < 1e-11 and er < 1e-11
    p.close()


def test_lih_cell_tabulated_element_matrices():
    """The LiH-like cell at full size with tabulated radials (48 samples per
    descriptor): the element matrices of the elements with the most local
    functions and of the most refined element against the oracle."""
    prob = W.with_tabulated_radials(W.lih_cell(), 48)
    say("tabulated lih_cell element matrices")
    o = oracle.Oracle(prob)
    p = P.Problem(prob).setup()
    xyz, _, qoff = p.quadrature()
    V = potential_at(xyz, prob)
    Vh = V.cpu().numpy()
    qoff = qoff.cpu().numpy()
    _, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    picks = sorted({int(np.argmax(nloc)), int(np.argmax(nleaf)), int(np.argmax(nloc * (nleaf > 1)))})
    for e in picks:
        He, Se = p.element_matrices(e, V)
        Ho, So = o.element_matrices(e, Vh[qoff[e]:qoff[e + 1]])
        eh, es = rel(He.cpu().numpy(), Ho), rel(Se.cpu().numpy(), So)
        say("element", e, "nloc", nloc[e], "leaves", nleaf[e], "H", eh, "S", es)
        assert eh < 1e-12 and es < 1e-12
    p.close()
