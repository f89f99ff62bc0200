"""GPU parity of the 32-node cubic serendipity elements (the paper's classical
FE, section "Self-consistent calculations") against the oracle, through the C
ABI: assembly (FP64 to 1e-12 and bf16x6 to 1e-7, at Gamma and general
k-points, including elements of more than 80 functions on the wide work
groups and wrapped cells), element matrices, the adjoint (1e-11), the
nonlocal term, tabulated radials on serendipity elements, and element
matrices of the LiH-like cell on a serendipity mesh at full size."""
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
    "lih": (lambda: W.small("lih", mesh=(2, 3, 2), fe_order=3, levels=1, n=4, a=5.0),
            [(0.0, 0.0, 0.0), (0.12, -0.24, 0.37)]),
    "one-wrap": (lambda: W.small("one", mesh=(3, 3, 2), fe_order=3, levels=2, n=3, a=4.6), [(0.31, 0.0, -0.2)]),
    "ceal-wide": (lambda: W.small("ceal", mesh=(2, 2, 2), fe_order=3, levels=1, n=3, a=4.4, rc=3.0, re=2.4),
                  [(0.0, 0.0, 0.0), (0.25, -0.25, 0.25)]),
    "lih-tabulated": (lambda: W.with_tabulated_radials(W.small("lih", mesh=(3, 2, 2), fe_order=3, levels=1, n=3,
                                                               a=5.0), 40), [(0.1, 0.2, -0.3)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_serendipity_assembly_matches_oracle(name):
    make, kpts = CASES[name]
    prob = make()
    say("serendipity assembly", name)
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    assert p.sizes["n_dof"] == o.n_dof and p.sizes["n_fe_slots"] == 7
    Vd = torch.from_numpy(V).cuda()
    H, S = p.assemble(Vd, kpts)
    Hs, Ss = p.assemble(Vd, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense(V, kap)
        eh = rel(p.to_dense(H[k]).cpu().numpy(), Ho)
        es = rel(p.to_dense(S[k]).cpu().numpy(), So)
        e6 = max(rel(p.to_dense(Hs[k]).cpu().numpy(), Ho), rel(p.to_dense(Ss[k]).cpu().numpy(), So))
        say(name, kap, "max n_loc", p.sizes["max_nloc"], "H", eh, "S", es, "bf16x6", e6)
        assert eh < 1e-12 and es < 1e-12 and e6 < 1e-7
    H2, S2 = p.assemble(Vd, kpts)
    assert torch.equal(H, H2) and torch.equal(S, S2)
    p.close()


def test_serendipity_element_matrices():
    prob = CASES["ceal-wide"][0]()
    say("serendipity element matrices")
    o = oracle.Oracle(prob)
    p = P.Problem(prob).setup()
    xyz, _, qoff = p.quadrature()
    V = potential_at(xyz, prob)
    Vh = V.cpu().numpy()
    qoff = qoff.cpu().numpy()
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    for e in sorted({int(np.argmax(nloc)), int(np.argmin(nloc)), 5}):
        He, Se = p.element_matrices(e, V)
        Ho, So = o.element_matrices(e, Vh[qoff[e]:qoff[e + 1]])
        eh, es = rel(He.cpu().numpy(), Ho), rel(Se.cpu().numpy(), So)
        say("element", e, "n_loc", nloc[e], "H", eh, "S", es)
        assert eh < 1e-12 and es < 1e-12
    p.close()


def test_serendipity_adjoint_matches_oracle():
    from test_gpu_backward import bsr_index
    prob = W.small("lih", mesh=(2, 3, 2), fe_order=3, levels=1, n=3, a=4.8, re=1.7, rc=2.1)
    say("serendipity adjoint")
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
    say("serendipity adjoint dL/dV", ev, "dL/dR", er)
    assert ev < 1e-11 and er < 1e-11
    p.close()


def test_serendipity_nonlocal_term():
    prob = W.with_projectors(W.small("lih", mesh=(3, 2, 2), fe_order=3, levels=1, n=3, a=5.0))
    say("serendipity nonlocal")
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    kap = (0.12, -0.24, 0.37)
    H, S = p.assemble(torch.from_numpy(V).cuda(), [kap])
    Ho, So = o.assemble_dense(V, kap)
    Vn = o.nonlocal_dense(kap)
    Hg = p.to_dense(H[0]).cpu().numpy()
    eh, en = rel(Hg, Ho + Vn), rel(Hg - Ho, Vn)
    say("serendipity nonlocal H", eh, "term", en)
    assert eh < 1e-12 and en < 1e-9 and rel(p.to_dense(S[0]).cpu().numpy(), So) < 1e-12
    p.close()


def test_lih_cell_serendipity_element_matrices():
    """The LiH-like cell (a = 7.6, 8^3 elements, 6^3 Gauss + 2 octree levels)
    on cubic serendipity elements: the element matrices of the elements with
    the most functions and of the most refined element against the oracle."""
    prob = dict(W.lih_cell(), fe_order=3, name="lih_cell_serendipity")
    say("serendipity lih_cell element matrices")
    o = oracle.Oracle(prob)
    p = P.Problem(prob).setup()
    xyz, _, qoff = p.quadrature()
    V = potential_at(xyz, prob)
    Vh = V.cpu().numpy()
    qoff = qoff.cpu().numpy()
    _, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    for e in sorted({int(np.argmax(nloc)), int(np.argmax(nleaf)), int(np.argmax(nloc * (nleaf > 1)))}):
        He, Se = p.element_matrices(e, V)
        Ho, So = o.element_matrices(e, Vh[qoff[e]:qoff[e + 1]])
        eh, es = rel(He.cpu().numpy(), Ho), rel(Se.cpu().numpy(), So)
        say("element", e, "n_loc", nloc[e], "leaves", nleaf[e], "H", eh, "S", es)
        assert eh < 1e-12 and es < 1e-12
    H, S = p.assemble(V, [(0.0, 0.0, 0.0)])
    assert torch.isfinite(H).all() and torch.isfinite(S).all()
    p.close()
