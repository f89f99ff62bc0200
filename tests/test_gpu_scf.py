"""GPU parity of the self-consistent field pieces (section "Self-consistent
calculations", eqs. poisson, veff, rhoe) against the oracle, through the C
ABI: the classical FE load vector and evaluation, the Hartree solve (small
cells and the LiH-like cell at full size), the LDA exchange-correlation, and
a few fixed-point iterations end to end."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1611_00731_amd as P  # noqa: E402
from paper_1611_00731_amd.scf import run_scf  # noqa: E402
from workloads.potential import potential_at  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def smooth_density(xyz, lat):
    """A positive, smooth, non-uniform density at Cartesian points."""
    u = xyz @ np.linalg.inv(np.asarray(lat))
    t = 2 * np.pi * u
    return 0.05 * (1.5 + np.cos(t[:, 0]) * np.sin(t[:, 1] + 0.3) + 0.4 * np.cos(2 * t[:, 2] - 0.7))


CASES = {
    "lih-p1": lambda: W.small("lih", mesh=(3, 2, 2), fe_order=1, levels=1, n=3, a=5.0),
    "lih-p2": lambda: W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0),
    "one-serendipity": lambda: W.small("one", mesh=(2, 3, 2), fe_order=3, levels=1, n=3, a=4.6),
    "one-skew": lambda: W.small("one", mesh=(2, 3, 2), fe_order=2, levels=0, n=4,
                                lattice=[[4.5, 0.3, -0.2], [0.1, 4.2, 0.25], [0.2, -0.3, 4.8]]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fe_load_eval_and_hartree_match_oracle(name):
    prob = CASES[name]()
    say("fe load/eval/hartree", name)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    n = smooth_density(xyz, prob["lattice"])
    p = P.Problem(prob).setup()
    assert p.sizes["n_vertex"] * p.sizes["n_fe_slots"] == o.n_fe_dof
    nd = torch.from_numpy(n).cuda()
    b = p.fe_load(nd).cpu().numpy()
    bo = o.fe_load(n)
    rng = np.random.default_rng(3)
    u = rng.normal(size=o.n_fe_dof)
    ev = p.fe_eval(torch.from_numpy(u).cuda()).cpu().numpy()
    evo = o.fe_eval(u)
    vh, v, it, res = p.hartree(nd)
    vho, vo = o.hartree(n)
    e = (rel(b, bo), rel(ev, evo), rel(v.cpu().numpy(), vo), rel(vh.cpu().numpy(), vho))
    say(name, "load", e[0], "eval", e[1], "hartree coefficients", e[2], "at points", e[3], "CG", it, res)
    assert e[0] < 1e-13 and e[1] < 1e-13 and e[2] < 1e-10 and e[3] < 1e-10 and res < 1e-13
    # a second solve reuses the stored operator and gives the same result
    vh2, _, _, _ = p.hartree(nd)
    assert torch.equal(vh, vh2)
    p.close()


def test_lda_matches_oracle():
    say("lda")
    rng = np.random.default_rng(4)
    rho = np.concatenate([10 ** rng.uniform(-6, 2, 4000), [0.0, -1.0, 3.0 / (4 * np.pi), 1e-31]])
    vo, eo = oracle.lda(rho)
    r = torch.from_numpy(rho).cuda()
    v = torch.empty_like(r)
    e = torch.empty_like(r)
    P.pufe_lda_xc(r, v, e)
    assert np.abs(v.cpu().numpy() - vo).max() < 1e-14 * np.abs(vo).max()
    assert np.abs(e.cpu().numpy() - eo).max() < 1e-14 * np.abs(eo).max()


def test_lih_cell_hartree_full_size():
    """The LiH-like cell at full size (4096 classical FE functions, 1.52 M
    points): the Hartree solve against the oracle's dense bordered solve."""
    prob = W.lih_cell()
    say("lih_cell hartree full size")
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    n = smooth_density(xyz, prob["lattice"])
    p = P.Problem(prob).setup()
    vh, v, it, res = p.hartree(torch.from_numpy(n).cuda())
    vho, vo = o.hartree(n)
    ev, ep = rel(v.cpu().numpy(), vo), rel(vh.cpu().numpy(), vho)
    say("lih_cell hartree: coefficients", ev, "at points", ep, "CG", it, res)
    assert ev < 1e-10 and ep < 1e-10
    p.close()


def test_scf_iterations_match_oracle():
    """Four fixed-point iterations (fig. scf) on a small LiH-like cell at two
    k-points: eigenvalues of every iteration and the final potential against
    the oracle's iteration."""
    prob = W.small("lih", mesh=(2, 2, 2), fe_order=1, levels=1, n=3, a=4.6,
                   kpts=((0.0, 0.0, 0.0), (0.25, 0.25, -0.25)))
    say("scf iterations")
    n_iter = 4
    Vo, ho = oracle.scf(prob, n_iter, alpha=0.3)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    p = P.Problem(prob).setup()
    V_ion = potential_at(torch.from_numpy(xyz).cuda(), prob)
    n_el = sum(prob["species_info"][s]["Z"] for s in prob["species"])
    V, h = run_scf(p, V_ion, n_el, prob["kpts"], n_iter, alpha=0.3)
    for i, ((e, r), (eo, ro)) in enumerate(zip(h, ho)):
        say("iteration", i, "eig diff", np.abs(e - eo).max(), "residual", r, ro)
        assert np.abs(e - eo).max() < 1e-8 and abs(r - ro) < 1e-8 * max(1.0, ro)
    assert rel(V.cpu().numpy(), Vo) < 1e-10
    assert ho[-1][1] < ho[0][1]
    p.close()


def test_lih_cell_density_full_size():
    """The LiH-like cell at full size (4888 DOFs) at Gamma: the dense
    eigenpairs are finite and their eigenvalues those of the eigenvalue-only
    solve; the density of the 8 doubly occupied states from the adjoint
    integrates to the 16 electrons; one fixed-point iteration gives a finite,
    positive residual."""
    from paper_1611_00731_amd.scf import bsr_index
    prob = W.lih_cell()
    say("lih_cell density full size")
    p = P.Problem(prob).setup()
    xyz, w, _ = p.quadrature()
    V = potential_at(xyz, prob)
    H, S = p.assemble(V, [(0.0, 0.0, 0.0)])
    Hd, Sd = p.to_dense(H[0]), p.to_dense(S[0])
    e, Cv = P.eigh(Hd, Sd)
    ev = P.eig(Hd, Sd, 16)
    assert torch.isfinite(torch.view_as_real(Cv)).all()
    assert float((e[:16] - ev).abs().max()) < 1e-9
    Co = Cv[:, :8]
    Pk = 2.0 * (Co @ Co.mH)
    r, c = bsr_index(p.layout())
    Pb = Pk[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()].contiguous()
    dV, _ = p.backward(V, (0.0, 0.0, 0.0), Pb, want_dR=False)
    n_e = float(dV.sum())
    say("electrons", n_e)
    assert abs(n_e - 16.0) < 1e-9
    _, hist = run_scf(p, V, 16.0, [(0.0, 0.0, 0.0)], 1)
    assert np.isfinite(hist[0][1]) and hist[0][1] > 0
    p.close()


def test_scf_smearing_matches_oracle():
    """Three fixed-point iterations with Fermi-Dirac smearing (width 0.02 Ha)
    on a small CeAl-like cell (15 electrons, s to f enrichments) at two
    k-points against the oracle's iteration."""
    prob = W.small("ceal", mesh=(2, 2, 2), fe_order=1, levels=1, n=3, a=4.4,
                   kpts=((0.0, 0.0, 0.0), (0.25, 0.25, -0.25)))
    say("scf smearing")
    n_iter = 3
    Vo, ho = oracle.scf(prob, n_iter, alpha=0.3, smearing=0.02)
    o = oracle.Oracle(prob)
    xyz, w, _ = o.quadrature()
    p = P.Problem(prob).setup()
    V_ion = potential_at(torch.from_numpy(xyz).cuda(), prob)
    n_el = sum(prob["species_info"][s]["Z"] for s in prob["species"])
    assert n_el == 15.0
    V, h = run_scf(p, V_ion, n_el, prob["kpts"], n_iter, alpha=0.3, smearing=0.02)
    for i, ((e, r), (eo, ro)) in enumerate(zip(h, ho)):
        say("iteration", i, "eig diff", np.abs(e - eo).max(), "residual", r, ro)
        assert np.abs(e - eo).max() < 1e-8 and abs(r - ro) < 1e-8 * max(1.0, ro)
    assert rel(V.cpu().numpy(), Vo) < 1e-10
    p.close()
