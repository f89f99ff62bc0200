"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Every case prints its name before touching the GPU.  Inputs are seeded and
synthetic; V is evaluated by the shared input generator at the oracle's
quadrature points (the canonical point order is the same on both sides).
Tolerance: relative Frobenius error <= 1e-12 for the FP64 path.
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

TOL = 1e-12


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_inputs(prob):
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    return o, xyz, w, off, V


def check_rule(p, o, xyz, w):
    lev, ijk, loff = P.pufe_get_leaves(p.ctx)
    olev, oijk, ooff = o.leaves()
    assert np.array_equal(loff, ooff)
    assert np.array_equal(lev, olev) and np.array_equal(ijk, oijk)
    gx, gw, goff = p.quadrature()
    assert np.array_equal(goff.cpu().numpy(), o.quadrature()[2])
    assert np.abs(gx.cpu().numpy() - xyz).max() < 1e-13 * max(1.0, np.abs(xyz).max())
    assert np.abs(gw.cpu().numpy() - w).max() < 1e-15 * max(1.0, w.max()) * 10


def _error_mode(prob, n=3, n_ref=6, levels=3, tol=1e-6):
    prob["quad"] = {"n": n, "n_ref": n_ref, "levels": levels, "mode": "error", "dist": 0.0, "tol": tol}
    return prob


SMALL = {
    "lih-error": (lambda: _error_mode(W.small("lih", mesh=(2, 2, 3), fe_order=2, a=4.8, re=1.6, rc=2.0)),
                  [(0.0, 0.0, 0.0), (0.1, -0.2, 0.3)]),
    "ceal-error": (lambda: _error_mode(W.small("ceal", mesh=(2, 2, 2), fe_order=1, a=4.4, rc=2.6, re=2.0),
                                       n=2, n_ref=4, levels=2, tol=1e-5), [(0.0, 0.0, 0.0)]),
    "single_atom_cube": (W.single_atom_cube, [(0.0, 0.0, 0.0), (0.1, 0.2, -0.3)]),
    "lih-p2-l1": (lambda: W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0),
                  [(0.0, 0.0, 0.0), (0.12, -0.24, 0.37), (0.25, 0.25, -0.25)]),
    "lih-odd-p1": (lambda: W.small("lih", mesh=(3, 3, 2), fe_order=1, levels=2, n=2, a=4.6),
                   [(0.31, 0.0, -0.2)]),
    "ceal-many": (lambda: W.small("ceal", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4,
                                  rc=3.0, re=2.4), [(0.0, 0.0, 0.0), (0.25, -0.25, 0.25)]),
    "one-skew": (lambda: W.small("one", mesh=(2, 3, 2), fe_order=2, levels=0, n=4,
                                 lattice=[[4.5, 0.3, -0.2], [0.1, 4.2, 0.25], [0.2, -0.3, 4.8]]),
                 [(0.1, 0.2, 0.3)]),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_assembly_matches_oracle(name):
    make, kpts = SMALL[name]
    prob = make()
    say("assembly", name, prob["mesh"], "p", prob["fe_order"])
    o, xyz, w, off, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    check_rule(p, o, xyz, w)
    Vd = torch.from_numpy(V).cuda()
    H, S = p.assemble(Vd, kpts)
    for k, kap in enumerate(kpts):
        Hg = p.to_dense(H[k]).cpu().numpy()
        Sg = p.to_dense(S[k]).cpu().numpy()
        Ho, So = o.assemble_dense(V, kap)
        assert rel(Hg, Ho) < TOL, (name, kap, rel(Hg, Ho))
        assert rel(Sg, So) < TOL, (name, kap, rel(Sg, So))
    # determinism: a second assembly is bitwise identical
    H2, S2 = p.assemble(Vd, kpts)
    assert torch.equal(H, H2) and torch.equal(S, S2)
    p.close()


def test_element_matrices_many_tiles():
    prob = SMALL["ceal-many"][0]()
    say("element matrices ceal-many")
    o, xyz, w, off, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    Vd = torch.from_numpy(V).cuda()
    nl = []
    for e in range(o.n_elem):
        He, Se = p.element_matrices(e, Vd)
        Ho, So = o.element_matrices(e, V[off[e]:off[e + 1]])
        nl.append(Ho.shape[0])
        assert rel(He.cpu().numpy(), Ho) < TOL and rel(Se.cpu().numpy(), So) < TOL
    assert max(nl) > 64 and min(nl) % 16 != 0   # several tile blocks and a ragged tail
    p.close()


def test_output_dtypes_gamma_and_c64():
    prob = SMALL["lih-p2-l1"][0]()
    say("output dtypes")
    o, xyz, w, off, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    Vd = torch.from_numpy(V).cuda()
    H, S = p.assemble(Vd, [(0, 0, 0)], out_dtype="c128")
    Hr, Sr = p.assemble(Vd, [(0, 0, 0)], out_dtype="f64")
    assert torch.equal(Hr[0], H[0, :, 0]) and torch.equal(Sr[0], S[0, :, 0])
    assert torch.count_nonzero(H[0, :, 1]) == 0
    kap = [(0.12, -0.24, 0.37)]
    H, S = p.assemble(Vd, kap, out_dtype="c128")
    Hf, Sf = p.assemble(Vd, kap, out_dtype="c64")
    assert rel(Hf.double().cpu().numpy(), H.cpu().numpy()) < 1e-6
    with pytest.raises(P.PufeError):
        p.assemble(Vd, kap, out_dtype="f64")
    p.close()


def test_single_atom_cube_eigenvalues():
    prob = W.single_atom_cube()
    say("single_atom_cube eigenvalues")
    o, xyz, w, off, V = oracle_inputs(prob)
    Ho, So = o.assemble_dense(V)
    ev_o = oracle.generalized_eigh(Ho, So, 4)
    p = P.Problem(prob).setup()
    H, S = p.assemble(torch.from_numpy(V).cuda())
    ev = P.eig(p.to_dense(H[0]), p.to_dense(S[0]), 4).cpu().numpy()
    assert np.abs(ev - ev_o).max() < 1e-9
    p.close()


def test_lih_cell_full_size_sampled_blocks():
    """The LiH-like workload at full size (512 elements, 1.52 M points): rule
    equality, and sampled BSR blocks (near and far from nuclei) against the
    oracle's block assembly."""
    prob = W.lih_cell()
    say("lih_cell full size")
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    p = P.Problem(prob).setup()
    check_rule(p, o, xyz, w)
    Vh = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    H, S = p.assemble(torch.from_numpy(Vh).cuda())
    lay = p.layout()
    Hh, Sh = H[0].cpu().numpy(), S[0].cpu().numpy()
    rng = np.random.default_rng(5)
    lev, _, loff = o.leaves()
    refined = [e for e in range(o.n_elem) if loff[e + 1] - loff[e] > 1]
    vs = [refined[0], refined[len(refined) // 2]] + list(rng.integers(0, o.n_vertex, 2))
    off_d = lay["dof_offset"]
    for v in vs:
        for kk in (lay["brow_ptr"][v], (lay["brow_ptr"][v] + lay["brow_ptr"][v + 1]) // 2):
            wv = int(lay["bcol"][kk])
            Hb, Sb = o.assemble_block(Vh, (0, 0, 0), int(v), wv)
            b0, b1 = lay["bval_offset"][kk], lay["bval_offset"][kk + 1]
            shape = (off_d[v + 1] - off_d[v], off_d[wv + 1] - off_d[wv])
            Hg = (Hh[b0:b1, 0] + 1j * Hh[b0:b1, 1]).reshape(shape)
            Sg = (Sh[b0:b1, 0] + 1j * Sh[b0:b1, 1]).reshape(shape)
            assert rel(Hg, Hb) < TOL and rel(Sg, Sb) < TOL, (v, wv)
    p.close()



# FP64 eigenvalue tolerance, from the reduction's rounding: the Cholesky
# reduction of H c = eps S c perturbs an eigenvalue by about
# u * kappa(S) * |eps| with u = 1.1e-16, kappa(S) ~ 1e7 for the enriched
# overlap and |eps| ~ 34 Ha here, i.e. ~4e-8 Ha, for the device solve and the
# LAPACK solve of the stored values alike.
EIG_TOL_FP64 = 1e-7


def test_lih_cell_eigenvalues_vs_oracle():
    """The LiH-like workload at full size: the lowest 16 eigenvalues of the
    FP64 GPU assembly against the FP64 oracle's (dense assembly and LAPACK
    solve, stored by tests/golden/make_lih_cell_eigenvalues.py)."""
    import os
    prob = W.lih_cell()
    say("lih_cell eigenvalues vs stored oracle eigenvalues")
    ev_o = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "lih_cell_eigenvalues.txt"), comments="#")
    assert len(ev_o) == prob["n_eig"]
    xyz, _, _ = oracle.Oracle(prob).quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    H, S = p.assemble(V)
    ev = P.eig(p.to_dense(H[0]).real.contiguous(), p.to_dense(S[0]).real.contiguous(), len(ev_o)).cpu().numpy()
    err = np.abs(ev - ev_o).max()
    say("max |eps - eps_oracle| (Ha)", err)
    assert err < EIG_TOL_FP64
    p.close()

def test_lih_cell_element_matrices_every_nloc():
    """Element matrices of the LiH-like workload at full size, one element per
    distinct n_loc (the most refined of each), against the oracle.  The set
    spans last tiles with at most 4 and with 5..8 real rows (the tail pairs
    of whole-element items) and fuller last tiles, on 3, 4 and 5 tiles."""
    prob = W.lih_cell()
    say("lih_cell element matrices, every n_loc")
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    Vh = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    p = P.Problem(prob).setup()
    Vd = torch.from_numpy(Vh).cuda()
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    nq = np.diff(off)
    picks = {}
    for e in range(o.n_elem):
        n = int(nloc[e])
        if n not in picks or nq[e] > nq[picks[n]]:
            picks[n] = e
    tails = {(n - 16 * ((n + 15) // 16 - 1)) for n in picks}
    assert any(t <= 4 for t in tails) and any(4 < t <= 8 for t in tails) and any(t > 8 for t in tails)
    for n, e in sorted(picks.items()):
        say("element", e, "n_loc", n, "points", int(nq[e]))
        He, Se = p.element_matrices(e, Vd)
        Ho, So = o.element_matrices(e, Vh[off[e]:off[e + 1]])
        assert rel(He.cpu().numpy(), Ho) < TOL, (e, n, rel(He.cpu().numpy(), Ho))
        assert rel(Se.cpu().numpy(), So) < TOL, (e, n, rel(Se.cpu().numpy(), So))
    p.close()


def test_ceal_cell_full_size_sampled():
    """The CeAl-like workload at full size (1728 elements, 27.3 M points,
    N = 37,891, n_loc up to 283: items of several row and column blocks):
    rule equality, element matrices of the unrefined element with the most
    functions and of the least refined octree element, and BSR blocks around
    vertices whose elements are all unrefined, at one k-point."""
    prob = W.ceal_cell()
    kap = tuple(prob["kpts"][1])
    say("ceal_cell full size")
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    p = P.Problem(prob).setup()
    check_rule(p, o, xyz, w)
    Vd = potential_at(torch.from_numpy(xyz).cuda(), prob)
    Vh = Vd.cpu().numpy()
    del xyz, w
    lev, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    plain = np.flatnonzero(nleaf == 1)
    refined = np.flatnonzero(nleaf > 1)
    e_big = int(plain[np.argmax(nloc[plain])])
    e_ref = int(refined[np.argmin(nleaf[refined])])
    say("ceal_cell elements", e_big, "n_loc", nloc[e_big], "|", e_ref, "leaves", nleaf[e_ref], "n_loc", nloc[e_ref])
    for e in (e_big, e_ref):
        He, Se = p.element_matrices(e, Vd)
        Ho, So = o.element_matrices(e, Vh[off[e]:off[e + 1]])
        assert rel(He.cpu().numpy(), Ho) < TOL and rel(Se.cpu().numpy(), So) < TOL, e
    H, S = p.assemble(Vd, [kap])
    lay = p.layout()
    Hh, Sh = H[0].cpu().numpy(), S[0].cpu().numpy()
    del H, S
    n1, n2, n3 = prob["mesh"]

    def all_plain(v):
        i, j, k = v % n1, (v // n1) % n2, v // (n1 * n2)
        return all(nleaf[((i - a) % n1) + n1 * (((j - b) % n2) + n2 * ((k - c) % n3))] == 1
                   for a in (0, 1) for b in (0, 1) for c in (0, 1))

    off_d = lay["dof_offset"]
    cand = [v for v in range(o.n_vertex) if all_plain(v)]
    width = np.diff(off_d)
    rng = np.random.default_rng(11)
    vs = [max(cand, key=lambda v: width[v])] + list(rng.choice(cand, 2, replace=False))
    for v in vs:
        v = int(v)
        for kk in (lay["brow_ptr"][v], lay["brow_ptr"][v + 1] - 1):
            wv = int(lay["bcol"][kk])
            if not all_plain(wv):
                continue
            Hb, Sb = o.assemble_block(Vh, kap, v, wv)
            b0, b1 = lay["bval_offset"][kk], lay["bval_offset"][kk + 1]
            shape = (off_d[v + 1] - off_d[v], off_d[wv + 1] - off_d[wv])
            Hg = (Hh[b0:b1, 0] + 1j * Hh[b0:b1, 1]).reshape(shape)
            Sg = (Sh[b0:b1, 0] + 1j * Sh[b0:b1, 1]).reshape(shape)
            say("ceal_cell block", v, wv, shape)
            assert rel(Hg, Hb) < TOL and rel(Sg, Sb) < TOL, (v, wv)
    p.close()


@pytest.mark.parametrize("p,mesh,kappa", [(1, (4, 3, 5), (0.1, -0.23, 0.37)),
                                           (2, (3, 2, 2), (0.12, -0.24, 0.37)),
                                           (2, (2, 3, 2), (0.0, 0.0, 0.0))])
def test_empty_lattice_closed_form(p, mesh, kappa):
    """The degenerate case with no enrichment (no groups, classical FE only)
    and V = 0: the lowest eigenvalues of the GPU assembly are sums of the 1D
    Bloch FE dispersions over the three axes, halved (the discrete |k+G|^2/2
    of an empty lattice), a closed form independent of the oracle."""
    from test_oracle_pins import _eig1d, bare, diag
    L = (3.0, 3.3, 2.7)
    prob = bare(diag(*L), mesh, p, n=3)
    say("empty lattice", p, mesh, kappa)
    pp = P.Problem(prob).setup()
    V = torch.zeros(pp.sizes["n_qp"], dtype=torch.float64, device="cuda")
    H, S = pp.assemble(V, [kappa])
    ev = P.eig(pp.to_dense(H[0]), pp.to_dense(S[0]), 12).cpu().numpy()
    lam = [_eig1d(mesh[d], L[d] / mesh[d], p, kappa[d]) for d in range(3)]
    allev = np.sort((lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]).ravel() / 2)
    assert np.abs(ev - allev[:12]).max() < 1e-11 * max(1, allev[11])
    pp.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_small_problems(seed):
    """Seeded random small problems (kind, mesh, element order, rule, cell
    shear, radii, two random k-points): the FP64 assembly against the oracle's
    dense assembly, the rule bit for bit, and the bf16x6 form to its bound."""
    prob = W.random_small(seed)
    say("random", seed, prob["mesh"], "p", prob["fe_order"], "levels", prob["quad"]["levels"],
        "n", prob["quad"]["n"], "atoms", len(prob["atoms"]))
    o, xyz, w, off, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    check_rule(p, o, xyz, w)
    Vd = torch.from_numpy(V).cuda()
    kpts = prob["kpts"]
    H, S = p.assemble(Vd, kpts)
    Hs, Ss = p.assemble(Vd, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense(V, kap)
        assert rel(p.to_dense(H[k]).cpu().numpy(), Ho) < TOL, (seed, kap)
        assert rel(p.to_dense(S[k]).cpu().numpy(), So) < TOL, (seed, kap)
        eh, es = rel(p.to_dense(Hs[k]).cpu().numpy(), Ho), rel(p.to_dense(Ss[k]).cpu().numpy(), So)
        say("bf16x6", seed, k, "H", eh, "S", es)
        assert eh < 1e-7 and es < 1e-7, (seed, kap)
    p.close()


def _golden_elements(path):
    """Checks of oracle element matrices stored by tests/golden/make_ceal_deep_elements.py."""
    out, cur = [], None
    for line in open(path):
        if line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "element":
            cur = {"e": int(vals[0]), "nloc": int(vals[1]), "nq": int(vals[2])}
            out.append(cur)
        elif key == "ab":
            cur["ab"] = np.array(vals, int).reshape(-1, 2)
        elif key.endswith("_fro"):
            cur[key] = float(vals[0])
        else:
            cur[key] = np.array(vals, float)
    return out


def _element_checks_error(c, M, name):
    """Largest relative error of the stored checks of one element matrix."""
    Mx = M @ c["x"]
    errs = [abs(np.linalg.norm(M) - c[name + "_fro"]) / c[name + "_fro"]]
    for got, ref in ((np.diag(M), c[name + "_diag"]), (Mx, c[name + "_x"]),
                     (M[c["ab"][:, 0], c["ab"][:, 1]], c[name + "_ab"])):
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return max(errs)


def test_ceal_cell_deepest_elements_fp64_and_split():
    """The CeAl-like workload at full size, deepest elements: the fully
    refined elements (262,144 and 147,456 points; hundreds of K-chunks,
    items of several row and column blocks) with the most local functions
    (283) and a fully refined element next to Al (99), against the oracle's
    element matrices stored by tests/golden/make_ceal_deep_elements.py, FP64
    (1e-12) and bf16x6 (1e-7); bf16x6 also on the unrefined element with the
    most functions and on BSR blocks around all-unrefined vertices against
    the oracle directly."""
    import os
    prob = W.ceal_cell()
    gold = _golden_elements(os.path.join(os.path.dirname(__file__), "golden", "ceal_deep_elements.txt"))
    say("ceal_cell deepest elements", [g["e"] for g in gold])
    p = P.Problem(prob).setup()
    xyz, _, qoff = p.quadrature()
    Vd = potential_at(xyz, prob)
    del xyz
    qoff = qoff.cpu().numpy()
    for prec, tol in (("fp64", TOL), ("bf16x6", 1e-7)):
        for g in gold:
            e = g["e"]
            assert qoff[e + 1] - qoff[e] == g["nq"]
            He, Se = p.element_matrices(e, Vd, precision=prec)
            assert He.shape[0] == g["nloc"]
            eh = _element_checks_error(g, He.cpu().numpy(), "H")
            es = _element_checks_error(g, Se.cpu().numpy(), "S")
            say(prec, "element", e, "H", eh, "S", es)
            assert eh < tol and es < tol, (prec, e, eh, es)
    # bf16x6 against the oracle on the largest unrefined element and on
    # blocks whose elements are all unrefined (same V array on both sides)
    o = oracle.Oracle(prob)
    _, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    plain = np.flatnonzero(nleaf == 1)
    e_big = int(plain[np.argmax(nloc[plain])])
    Vh = Vd.cpu().numpy()
    He, Se = p.element_matrices(e_big, Vd, precision="bf16x6")
    Ho, So = o.element_matrices(e_big, Vh[qoff[e_big]:qoff[e_big + 1]])
    say("bf16x6 element", e_big, "H", rel(He.cpu().numpy(), Ho), "S", rel(Se.cpu().numpy(), So))
    assert rel(He.cpu().numpy(), Ho) < 1e-7 and rel(Se.cpu().numpy(), So) < 1e-7
    kap = tuple(prob["kpts"][2])
    H, S = p.assemble(Vd, [kap], precision="bf16x6")
    lay = p.layout()
    Hh, Sh = H[0].cpu().numpy(), S[0].cpu().numpy()
    del H, S
    n1, n2, n3 = prob["mesh"]

    def all_plain(v):
        i, j, k = v % n1, (v // n1) % n2, v // (n1 * n2)
        return all(nleaf[((i - a) % n1) + n1 * (((j - b) % n2) + n2 * ((k - c) % n3))] == 1
                   for a in (0, 1) for b in (0, 1) for c in (0, 1))

    off_d = lay["dof_offset"]
    width = np.diff(off_d)
    cand = [v for v in range(o.n_vertex) if all_plain(v)]
    rng = np.random.default_rng(12)
    for v in [max(cand, key=lambda v: width[v])] + list(rng.choice(cand, 2, replace=False)):
        v = int(v)
        kk = lay["brow_ptr"][v]
        wv = int(lay["bcol"][kk])
        if not all_plain(wv):
            continue
        Hb, Sb = o.assemble_block(Vh, kap, v, wv)
        b0, b1 = lay["bval_offset"][kk], lay["bval_offset"][kk + 1]
        shape = (off_d[v + 1] - off_d[v], off_d[wv + 1] - off_d[wv])
        Hg = (Hh[b0:b1, 0] + 1j * Hh[b0:b1, 1]).reshape(shape)
        Sg = (Sh[b0:b1, 0] + 1j * Sh[b0:b1, 1]).reshape(shape)
        say("bf16x6 block", v, wv, shape, rel(Hg, Hb), rel(Sg, Sb))
        assert rel(Hg, Hb) < 1e-7 and rel(Sg, Sb) < 1e-7, (v, wv)
    p.close()


def _rule_cells(lev, ijk, loff):
    """Leaves and internal cells of every element's octree, as sets of (e, level, c1, c2, c3)."""
    leaves, internal = set(), set()
    for e in range(len(loff) - 1):
        for k in range(loff[e], loff[e + 1]):
            l, c = int(lev[k]), tuple(int(x) for x in ijk[k])
            leaves.add((e, l) + c)
            for up in range(1, l + 1):
                internal.add((e, l - up) + tuple(x >> up for x in c))
    return leaves, internal


# Tie margin of the error-driven rule: two implementations may decide a cell
# differently only where one of its error estimates |Q_n - Q_ref| lies within
# this absolute distance of the tolerance (the estimates are differences of
# O(1) sums and agree to ~1e-15 between the two).
RULE_TIE = 1e-9


ERROR_CASES = {
    "lih-error": SMALL["lih-error"],
    "ceal-error": SMALL["ceal-error"],
    # the paper's triclinic CeAl cell (skewed element maps) at a small mesh
    "ceal-triclinic": (lambda: W.ceal_triclinic(mesh=3, levels=2, n=3, n_ref=5, tol=1e-4), W.PAPER_KPTS),
}


@pytest.mark.parametrize("name", sorted(ERROR_CASES))
def test_error_rule_ties_and_assembly_on_one_shared_rule(name):
    """The error-driven rule (section "Adaptive quadrature") built on the GPU
    against the oracle's: any cell decided differently must be a tie (an
    error estimate within RULE_TIE of the tolerance); then the library
    assembles on the oracle's own rule (pufe_set_rule) and H, S match the
    oracle at 1e-12."""
    from test_oracle_pins_rule import _cell_errors, _element_functions
    make, kpts = ERROR_CASES[name]
    prob = make()
    q = prob["quad"]
    say("error rule ties + shared rule", name)
    o, xyz, w, off, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    glev, gijk, goff = P.pufe_get_leaves(p.ctx)
    olev, oijk, ooff = o.leaves()
    gl, gi = _rule_cells(glev, gijk, goff)
    ol, oi = _rule_cells(olev, oijk, ooff)
    decided = (gl & oi) | (ol & gi)   # a leaf in one rule, split in the other
    for (e, l, *c) in sorted(decided):
        near = min(min(abs(x - q["tol"]) for x in _cell_errors(o, prob, e, l, c, fn, q["n"], q["n_ref"]))
                   for fn in _element_functions(o, prob, e))
        assert near <= RULE_TIE, (name, e, l, c, near)
    say("cells decided differently", len(decided))
    p.set_rule(olev, oijk, ooff)
    assert p.sizes["n_qp"] == o.n_qp
    Vd = torch.from_numpy(V).cuda()
    for kap in kpts:
        Ho, So = o.assemble_dense(V, kap)
        for prec, tol in (("fp64", TOL), ("bf16x6", 1e-7)):
            H, S = p.assemble(Vd, [kap], precision=prec)
            eh, es = rel(p.to_dense(H[0]).cpu().numpy(), Ho), rel(p.to_dense(S[0]).cpu().numpy(), So)
            say(name, prec, kap, "H", eh, "S", es)
            assert eh < tol and es < tol, (prec, kap)
    # a malformed rule is refused: drop one leaf of the first element
    with pytest.raises(P.PufeError):
        bad = ooff.copy()
        bad[1:] -= 1
        P.pufe_set_rule(p.ctx, np.delete(olev, 0), np.delete(oijk, 0, axis=0), bad)
    p.close()
