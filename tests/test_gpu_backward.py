"""GPU parity of the adjoint (assemble_backward) and its autograd wrapper.

dL/dV is compared with the oracle point by point; dL/dR with the oracle on
small cases and with central finite differences (h = 1e-4 bohr) of the GPU
forward, rule and enriched sets frozen, at the 64-atom supercell size; the
split-precision forms likewise, to the bounds their limbs allow.
"""
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


def bsr_index(lay):
    """Global (row, col) DOF of every stored BSR entry, in value order."""
    off, rp, bc, bo = lay["dof_offset"], lay["brow_ptr"], lay["bcol"], lay["bval_offset"]
    rows, cols = [], []
    for v in range(len(rp) - 1):
        bv = off[v + 1] - off[v]
        for k in range(rp[v], rp[v + 1]):
            w = bc[k]
            bw = off[w + 1] - off[w]
            r = np.repeat(np.arange(off[v], off[v + 1]), bw)
            c = np.tile(np.arange(off[w], off[w + 1]), bv)
            rows.append(r)
            cols.append(c)
    return np.concatenate(rows), np.concatenate(cols)


def small_case():
    prob = W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=4.8, re=1.7, rc=2.1)
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    Cp = W.adjoint_factor(o.n_dof, rank=6, seed=0)
    Cq = W.adjoint_factor(o.n_dof, rank=3, seed=1)
    return prob, o, V, Cp @ Cp.conj().T, Cq @ Cq.conj().T


def test_backward_matches_oracle_small():
    prob, o, V, Pd, Qd = small_case()
    kap = (0.12, -0.24, 0.37)
    say("backward small vs oracle")
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    Vd = torch.from_numpy(V).cuda()
    dV, dR = p.backward(Vd, kap, Pb, Qb)
    assert rel(dV.cpu().numpy(), dV_o) < 1e-11
    assert np.abs(dR.cpu().numpy() - dR_o).max() < 1e-11 * np.abs(dR_o).max()
    # P only and Q only add up to both
    dV1, dR1 = p.backward(Vd, kap, Pb, None)
    dV2, dR2 = p.backward(Vd, kap, None, Qb)
    assert torch.equal(dV1, dV) and torch.count_nonzero(dV2) == 0
    assert torch.allclose(dR1 + dR2, dR, rtol=0, atol=1e-13 * float(dR.abs().max()))
    # repeated calls are bitwise identical
    dV3, dR3 = p.backward(Vd, kap, Pb, Qb)
    assert torch.equal(dV3, dV) and torch.equal(dR3, dR)
    p.close()


def test_autograd_function_and_finite_differences():
    prob, o, V, Pd, Qd = small_case()
    kap = (0.25, 0.0, -0.13)
    say("autograd + FD small")
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    Fn = P.PUFEAssemble()
    R0 = np.asarray(prob["atoms"], float)
    Vt = torch.from_numpy(V).cuda().requires_grad_(True)
    Rt = torch.tensor(R0, dtype=torch.float64, requires_grad=True)
    H, S = Fn.apply(p, Vt, Rt, kap)
    L = (Pb.conj() * H).real.sum() + (Qb.conj() * S).real.sum()
    L.backward()
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    assert rel(Vt.grad.cpu().numpy(), dV_o) < 1e-11
    assert np.abs(Rt.grad.cpu().numpy() - dR_o).max() < 1e-11 * np.abs(dR_o).max()

    def loss(R):
        p.set_positions(R)
        with torch.no_grad():
            H, S = p.assemble(torch.from_numpy(V).cuda(), [kap])
        Hc = torch.view_as_complex(H[0])
        Sc = torch.view_as_complex(S[0])
        return float((Pb.conj() * Hc).real.sum() + (Qb.conj() * Sc).real.sum())

    h = 1e-4
    g = Rt.grad.cpu().numpy()
    for A, k in [(0, 0), (1, 2), (5, 1), (6, 0)]:
        Rp, Rm = R0.copy(), R0.copy()
        Rp[A, k] += h
        Rm[A, k] -= h
        fd = (loss(Rp) - loss(Rm)) / (2 * h)
        assert abs(fd - g[A, k]) < 1e-6 * max(1.0, np.abs(g).max()), (A, k, fd, g[A, k])
    p.set_positions(R0)
    p.close()


def _golden_supercell():
    import os
    dR, dVs = {}, {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "lih_supercell_adjoint.txt")):
        if line.startswith("#"):
            continue
        key, idx, *vals = line.split()
        if key == "dLdR":
            dR[int(idx)] = [float(v) for v in vals]
        else:
            dVs[int(idx)] = float(vals[0])
    return np.array([dR[A] for A in sorted(dR)]), np.array([dVs[e] for e in sorted(dVs)])


def test_backward_lih_supercell_full_size():
    """2x2x2 LiH-like supercell (64 atoms, 4096 elements, 12.1 M points),
    rank-128 Hermitian PSD P on the pattern: dL/dR of all 64 atoms and dL/dV
    summed over the points of every element against the oracle's full adjoint
    (stored by tests/golden/make_lih_supercell_adjoint.py), FP64 and bf16x6;
    dL/dV point by point on sampled elements against the oracle's
    per-element adjoint; dL/dR against central differences of the GPU
    forward on all 192 coordinates."""
    prob = W.lih_supercell()
    say("backward lih_supercell full size")
    gR, gVs = _golden_supercell()
    o = oracle.Oracle(prob)
    xyz, w, qoff = o.quadrature()
    Vd = potential_at(torch.from_numpy(xyz).cuda(), prob)
    V = Vd.cpu().numpy()
    del xyz, w
    p = P.Problem(prob).setup()
    lay = p.layout()
    N = p.sizes["n_dof"]
    Cf = W.adjoint_factor(N, rank=128, seed=0)
    Cd = torch.from_numpy(Cf).cuda()
    rows, cols = bsr_index(lay)
    rows_d = torch.from_numpy(rows).cuda()
    cols_d = torch.from_numpy(cols).cuda()
    Pb = torch.empty(len(rows), dtype=torch.complex128, device="cuda")
    for s in range(0, len(rows), 1 << 20):
        r, c = rows_d[s:s + (1 << 20)], cols_d[s:s + (1 << 20)]
        Pb[s:s + (1 << 20)] = (Cd[r] * Cd[c].conj()).sum(-1)
    del Cd, rows_d, cols_d
    qo = torch.from_numpy(qoff).cuda()
    seg = torch.repeat_interleave(torch.arange(len(qoff) - 1, device="cuda"), qo[1:] - qo[:-1])

    def elem_sums(dV):
        return torch.zeros(len(qoff) - 1, dtype=torch.float64, device="cuda").index_add_(0, seg, dV).cpu().numpy()

    dV, dR = p.backward(Vd, (0.0, 0.0, 0.0), Pb, None)
    g = dR.cpu().numpy()
    eR = np.abs(g - gR).max() / np.abs(gR).max()
    eV = np.abs(elem_sums(dV) - gVs).max() / np.abs(gVs).max()
    say("fp64 vs oracle: dL/dR", eR, "dL/dV element sums", eV)
    assert eR < 1e-11 and eV < 1e-11
    dVh = dV.cpu().numpy()
    lev, _, loff = o.leaves()
    refined = [e for e in range(o.n_elem) if loff[e + 1] - loff[e] > 1]
    for e in [refined[0], refined[len(refined) // 2], 5, 1234, o.n_elem - 1]:
        gd, _ = o.element_dofs(e)
        Ploc = Cf[gd] @ Cf[gd].conj().T
        dv_o, _ = o.backward_element(e, V[qoff[e]:qoff[e + 1]], (0, 0, 0), Ploc)
        assert rel(dVh[qoff[e]:qoff[e + 1]], dv_o) < 1e-11, e
    # the split form at full size (bf16x6) against the same oracle values
    dVs, dRs = p.backward(Vd, (0.0, 0.0, 0.0), Pb, None, precision="bf16x6")
    eRs = np.abs(dRs.cpu().numpy() - gR).max() / np.abs(gR).max()
    eVs = rel(dVs.cpu().numpy(), dVh)
    say("bf16x6: dL/dR vs oracle", eRs, "dL/dV vs FP64", eVs)
    assert eRs < SPLIT_TOL["bf16x6"] and eVs < SPLIT_TOL["bf16x6"]
    R0 = np.asarray(prob["atoms"], float)

    def loss(R):
        p.set_positions(R)
        H, _ = p.assemble(Vd, [(0, 0, 0)], with_S=False)
        return float((Pb.conj() * torch.view_as_complex(H[0])).real.sum())

    h = 1e-4
    worst = 0.0
    for A in range(len(R0)):
        for k in range(3):
            Rp, Rm = R0.copy(), R0.copy()
            Rp[A, k] += h
            Rm[A, k] -= h
            fd = (loss(Rp) - loss(Rm)) / (2 * h)
            worst = max(worst, abs(fd - g[A, k]) / np.abs(g).max())
    say("central differences, all 192 coordinates: worst relative error", worst)
    assert worst < 1e-6
    p.set_positions(R0)
    p.close()


# Split-precision adjoint tolerances (relative): U = Ps B is summed from the
# kept bf16 limb products in FP32, which leaves about 2^-24 per product with
# three limbs (the FP32 sums) and about 3 * 2^-18 with two (the dropped
# limb products and residuals); the bounds allow ten times that for the sums.
SPLIT_TOL = {"bf16x6": 1e-6, "bf16x3": 1e-4}


@pytest.mark.parametrize("prec", ["bf16x6", "bf16x3"])
def test_backward_split_matches_oracle_small(prec):
    """Split-precision adjoint (bf16 limbs of Ps and of the basis rows on the
    BF16 MFMAs) against the FP64 oracle: dL/dV and dL/dR, P and Q passes."""
    prob, o, V, Pd, Qd = small_case()
    kap = (0.12, -0.24, 0.37)
    say("backward split small vs oracle", prec)
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    dV, dR = p.backward(torch.from_numpy(V).cuda(), kap, Pb, Qb, precision=prec)
    ev = rel(dV.cpu().numpy(), dV_o)
    er = np.abs(dR.cpu().numpy() - dR_o).max() / np.abs(dR_o).max()
    say(prec, "dL/dV", ev, "dL/dR", er)
    assert ev < SPLIT_TOL[prec] and er < SPLIT_TOL[prec]
    p.close()


@pytest.mark.parametrize("seed", [0, 3, 4, 7])
def test_backward_random_small_problems(seed):
    """The adjoint on seeded random small problems (elements of at most 80
    functions), FP64 and bf16x6, against the oracle at a random k-point."""
    prob = W.random_small(seed)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    Cp = W.adjoint_factor(o.n_dof, rank=5, seed=seed)
    Cq = W.adjoint_factor(o.n_dof, rank=2, seed=seed + 100)
    Pd, Qd = Cp @ Cp.conj().T, Cq @ Cq.conj().T
    kap = prob["kpts"][1]
    say("backward random", seed, prob["mesh"], "p", prob["fe_order"], "k", kap)
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    Vd = torch.from_numpy(V).cuda()
    for prec, tol in (("fp64", 1e-11), ("bf16x6", SPLIT_TOL["bf16x6"])):
        dV, dR = p.backward(Vd, kap, Pb, Qb, precision=prec)
        ev = rel(dV.cpu().numpy(), dV_o)
        er = np.abs(dR.cpu().numpy() - dR_o).max() / np.abs(dR_o).max()
        say(prec, "dL/dV", ev, "dL/dR", er)
        assert ev < tol and er < tol, (seed, prec)
    p.close()


WIDE_CASES = {
    # 16 of 18 elements above 80 functions (up to 132: three row blocks)
    "ceal-mixed": lambda: W.small("ceal", mesh=(3, 3, 2), fe_order=2, levels=1, n=3, a=5.4, rc=3.0, re=2.0),
    # serendipity elements of up to 196 functions (four row blocks)
    "ceal-serendipity": lambda: W.small("ceal", mesh=(2, 2, 2), fe_order=3, levels=1, n=3, a=4.4, rc=3.0, re=2.4),
}


@pytest.mark.parametrize("name", sorted(WIDE_CASES))
def test_backward_wide_elements_match_oracle(name):
    """Elements of more than 80 functions (the block of Ps streamed through
    LDS in 64 x 64 blocks): dL/dV and dL/dR against the oracle's dense
    adjoint at a general k-point, P and Q both given; the split forms refuse
    such elements."""
    prob = WIDE_CASES[name]()
    say("backward wide elements", name)
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    Cp = W.adjoint_factor(o.n_dof, rank=6, seed=0)
    Cq = W.adjoint_factor(o.n_dof, rank=3, seed=1)
    Pd, Qd = Cp @ Cp.conj().T, Cq @ Cq.conj().T
    kap = (0.12, -0.24, 0.37)
    dV_o, dR_o = o.backward_dense(V, kap, Pd, Qd)
    p = P.Problem(prob).setup()
    rows, cols = bsr_index(p.layout())
    Pb = torch.from_numpy(Pd[rows, cols]).cuda()
    Qb = torch.from_numpy(Qd[rows, cols]).cuda()
    Vd = torch.from_numpy(V).cuda()
    dV, dR = p.backward(Vd, kap, Pb, Qb)
    ev = rel(dV.cpu().numpy(), dV_o)
    er = np.abs(dR.cpu().numpy() - dR_o).max() / np.abs(dR_o).max()
    say(name, "max n_loc", p.sizes["max_nloc"], "dL/dV", ev, "dL/dR", er)
    assert p.sizes["max_nloc"] > 80 and ev < 1e-11 and er < 1e-11
    dV2, dR2 = p.backward(Vd, kap, Pb, Qb)
    assert torch.equal(dV2, dV) and torch.equal(dR2, dR)
    with pytest.raises(P.PufeError) as err:
        p.backward(Vd, kap, Pb, Qb, precision="bf16x6")
    assert err.value.code == -2
    p.close()


def test_backward_ceal_cell_full_size():
    """The CeAl-like cell (1728 elements, 27.3 M points, n_loc up to 283) with
    a rank-16 Hermitian PSD P on the pattern at Gamma: dL/dV point by point
    on sampled elements (refined and not, above 80 functions) against the
    oracle's per-element adjoint, and dL/dR of both atoms against central
    differences of the GPU forward."""
    prob = W.ceal_cell()
    say("backward ceal_cell full size")
    o = oracle.Oracle(prob)
    p = P.Problem(prob).setup()
    xyz, _, qoff = p.quadrature()
    Vd = potential_at(xyz, prob)
    del xyz
    qoff = qoff.cpu().numpy()
    lay = p.layout()
    N = p.sizes["n_dof"]
    Cf = W.adjoint_factor(N, rank=16, seed=2)
    Cd = torch.from_numpy(Cf).cuda()
    rows, cols = bsr_index(lay)
    Pb = torch.empty(len(rows), dtype=torch.complex128, device="cuda")
    for s in range(0, len(rows), 1 << 22):
        r = torch.from_numpy(rows[s:s + (1 << 22)]).cuda()
        c = torch.from_numpy(cols[s:s + (1 << 22)]).cuda()
        Pb[s:s + (1 << 22)] = (Cd[r] * Cd[c].conj()).sum(-1)
    del Cd
    dV, dR = p.backward(Vd, (0.0, 0.0, 0.0), Pb, None)
    dVh = dV.cpu().numpy()
    g = dR.cpu().numpy()
    _, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    wide = np.nonzero(nloc > 80)[0]
    picks = [int(wide[np.argmax(nloc[wide] * (nleaf[wide] == 1))]),                     # widest unrefined
             int(wide[np.argmin(np.where(nleaf[wide] > 1, nleaf[wide], 1 << 30))]),     # least refined wide
             int(np.argmin(nloc))]                                                        # a narrow one
    Vh = Vd.cpu().numpy()
    for e in picks:
        gd, _ = o.element_dofs(e)
        Ploc = Cf[gd] @ Cf[gd].conj().T
        dv_o, _ = o.backward_element(e, Vh[qoff[e]:qoff[e + 1]], (0, 0, 0), Ploc)
        err = rel(dVh[qoff[e]:qoff[e + 1]], dv_o)
        say("element", e, "n_loc", nloc[e], "leaves", nleaf[e], "dL/dV", err)
        assert err < 1e-11
    R0 = np.asarray(prob["atoms"], float)

    def loss(R):
        p.set_positions(R)
        H, _ = p.assemble(Vd, [(0, 0, 0)], with_S=False)
        return float((Pb.conj() * torch.view_as_complex(H[0])).real.sum())

    h = 1e-4
    worst = 0.0
    for A in range(len(R0)):
        for k in range(3):
            Rp, Rm = R0.copy(), R0.copy()
            Rp[A, k] += h
            Rm[A, k] -= h
            fd = (loss(Rp) - loss(Rm)) / (2 * h)
            worst = max(worst, abs(fd - g[A, k]) / np.abs(g).max())
    say("ceal dL/dR", g.tolist(), "central differences worst relative error", worst)
    assert worst < 1e-6
    p.set_positions(R0)
    p.close()
