"""GPU parity of the Bloch-periodic enrichment (eq. Psi with f(R) = exp(i k.R);
periodic PU, boundary phases on the classical FE) against the oracle, through
the C ABI.  The library contracts, per k-point, the real and imaginary rows of
every enriched function on the real MFMA path and forms the complex element
matrices in the scatter; the oracle integrates conj(phi_a) phi_b directly.

Tolerances as for the periodic form: relative Frobenius error <= 1e-12 in
FP64 and <= 1e-7 for bf16x6."""
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
KAP = (0.12, -0.24, 0.37)


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def oracle_inputs(prob):
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    return o, V


B = W.with_bloch_enrichment
CASES = {
    # one atom, images overlapping (rc 3.0 in a 4.6 cell), trilinear FE
    "one-overlap-p1": (lambda: B(W.small("one", mesh=(3, 3, 2), fe_order=1, levels=1, n=3, a=4.6, rc=3.0, re=2.4)),
                       [(0.0, 0.0, 0.0), (0.31, -0.17, 0.23)]),
    # LiH-like cell, triquadratic FE, mesh of odd and even sizes
    "lih-p2": (lambda: B(W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)),
               [KAP, (0.25, 0.25, -0.25), (0.5, 0.0, 0.0)]),
    # elements of 219 rows (wide work items, several row and column blocks)
    "lih-p2-wide": (lambda: B(W.small("lih", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4, re=2.4, rc=2.8)),
                    [KAP]),
    # serendipity FE, tabulated radials
    "one-serendipity": (lambda: B(W.small("one", mesh=(2, 3, 2), fe_order=3, levels=1, n=3, a=4.6, rc=3.0, re=2.0)),
                        [(0.2, 0.1, -0.4)]),
    "lih-tabulated": (lambda: B(W.with_tabulated_radials(W.small("lih", mesh=(3, 2, 2), fe_order=1, levels=1, n=3,
                                                                 a=5.0), 40)), [(0.1, 0.2, -0.3)]),
    # skewed cell
    "one-skew": (lambda: B(W.small("one", mesh=(2, 3, 2), fe_order=2, levels=0, n=4,
                                   lattice=[[4.5, 0.3, -0.2], [0.1, 4.2, 0.25], [0.2, -0.3, 4.8]])),
                 [(0.1, 0.2, 0.3)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_bloch_assembly_matches_oracle(name):
    make, kpts = CASES[name]
    prob = make()
    say("bloch assembly", name)
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    assert p.sizes["n_dof"] == o.n_dof
    Vd = torch.from_numpy(V).cuda()
    H, S = p.assemble(Vd, kpts)
    H6, S6 = p.assemble(Vd, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense_bloch(V, kap)
        Hg, Sg = p.to_dense(H[k]).cpu().numpy(), p.to_dense(S[k]).cpu().numpy()
        eh, es = rel(Hg, Ho), rel(Sg, So)
        e6 = max(rel(p.to_dense(H6[k]).cpu().numpy(), Ho), rel(p.to_dense(S6[k]).cpu().numpy(), So))
        say(name, kap, "rows", p.sizes["max_nloc"], "H", eh, "S", es, "bf16x6", e6)
        assert eh < TOL and es < TOL and e6 < 1e-7
    H2, S2 = p.assemble(Vd, kpts)
    assert torch.equal(H, H2) and torch.equal(S, S2)
    p.close()


def test_bloch_gamma_output_types_and_many_kpoints():
    """At Gamma the Bloch form equals the periodic form; real (f64) and c64
    outputs; more k-points in one call than one phase table holds (16), each
    equal to its single-k assembly."""
    prob = CASES["lih-p2"][0]()
    say("bloch gamma, dtypes, 18 k-points")
    o, V = oracle_inputs(prob)
    Vd = torch.from_numpy(V).cuda()
    p = P.Problem(prob).setup()
    per = dict(prob)
    per.pop("enrichment_phase")
    q = P.Problem(per).setup()
    Hb, Sb = p.assemble(Vd, [(0, 0, 0)])
    Hp, Sp = q.assemble(Vd, [(0, 0, 0)])
    assert rel(Hb.cpu().numpy(), Hp.cpu().numpy()) < TOL and rel(Sb.cpu().numpy(), Sp.cpu().numpy()) < TOL
    assert torch.count_nonzero(Hb[0, :, 1]) == 0
    Hr, Sr = p.assemble(Vd, [(0, 0, 0)], out_dtype="f64")
    assert torch.equal(Hr[0], Hb[0, :, 0]) and torch.equal(Sr[0], Sb[0, :, 0])
    Hc, Sc = p.assemble(Vd, [KAP], out_dtype="c128")
    Hf, Sf = p.assemble(Vd, [KAP], out_dtype="c64")
    assert rel(Hf.double().cpu().numpy(), Hc.cpu().numpy()) < 1e-6
    assert rel(Sf.double().cpu().numpy(), Sc.cpu().numpy()) < 1e-6
    rng = np.random.default_rng(7)
    kpts = [tuple(k) for k in rng.uniform(-0.5, 0.5, (18, 3))]
    Hm, Sm = p.assemble(Vd, kpts)
    for k in (0, 15, 16, 17):
        H1, S1 = p.assemble(Vd, [kpts[k]])
        assert torch.equal(Hm[k], H1[0]) and torch.equal(Sm[k], S1[0]), k
    Ho, So = o.assemble_dense_bloch(V, kpts[17])
    assert rel(p.to_dense(Hm[17]).cpu().numpy(), Ho) < TOL
    p.close()
    q.close()


def test_bloch_unsupported_entries():
    prob = CASES["one-overlap-p1"][0]()
    say("bloch unsupported entries")
    o, V = oracle_inputs(prob)
    Vd = torch.from_numpy(V).cuda()
    p = P.Problem(prob).setup()
    nnz = p.sizes["nnz"]
    H = torch.empty((1, nnz, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PufeError) as ei:
        P.pufe_assemble_noalloc(p.ctx, Vd, [KAP], "fp64", "c128", H, None)
    assert ei.value.code == -2
    with pytest.raises(P.PufeError) as ei:
        p.element_matrices(0, Vd)
    assert ei.value.code == -2
    Pz = torch.zeros((nnz, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PufeError) as ei:
        p.backward(Vd, KAP, Pz)
    assert ei.value.code == -2
    with pytest.raises(P.PufeError) as ei:
        P.Batch([p])
    assert ei.value.code == -5 or ei.value.code == -2
    p.close()


def test_lih_cell_bloch_full_size_sampled_blocks():
    """The LiH-like workload at full size (512 elements, 1.52 M points, up to
    107 rows per element) with Bloch-periodic enrichment at a general k-point:
    sampled BSR blocks near and far from nuclei against the oracle's block
    assembly, FP64 and bf16x6."""
    prob = B(W.lih_cell())
    say("lih_cell bloch full size")
    o = oracle.Oracle(prob)
    xyz, w, off = o.quadrature()
    p = P.Problem(prob).setup()
    Vh = potential_at(torch.from_numpy(xyz).cuda(), prob).cpu().numpy()
    Vd = torch.from_numpy(Vh).cuda()
    H, S = p.assemble(Vd, [KAP])
    H6, S6 = p.assemble(Vd, [KAP], precision="bf16x6")
    lay = p.layout()
    Hh, Sh, H6h, S6h = H[0].cpu().numpy(), S[0].cpu().numpy(), H6[0].cpu().numpy(), S6[0].cpu().numpy()
    rng = np.random.default_rng(5)
    _, _, loff = o.leaves()
    refined = [e for e in range(o.n_elem) if loff[e + 1] - loff[e] > 1]
    vs = [refined[0], refined[len(refined) // 2]] + list(rng.integers(0, o.n_vertex, 2))
    off_d = lay["dof_offset"]
    for v in vs:
        for kk in (lay["brow_ptr"][v], (lay["brow_ptr"][v] + lay["brow_ptr"][v + 1]) // 2):
            wv = int(lay["bcol"][kk])
            Hb, Sb = o.assemble_block_bloch(Vh, KAP, int(v), wv)
            b0, b1 = lay["bval_offset"][kk], lay["bval_offset"][kk + 1]
            shape = (off_d[v + 1] - off_d[v], off_d[wv + 1] - off_d[wv])

            def blk(A):
                return (A[b0:b1, 0] + 1j * A[b0:b1, 1]).reshape(shape)

            eh, es = rel(blk(Hh), Hb), rel(blk(Sh), Sb)
            e6 = max(rel(blk(H6h), Hb), rel(blk(S6h), Sb))
            say("block", int(v), wv, "H", eh, "S", es, "bf16x6", e6)
            assert eh < TOL and es < TOL and e6 < 1e-7, (v, wv)
    p.close()


def test_bloch_error_rule():
    """Error-driven rule with the Bloch-periodic enrichment: the library
    builds the same rule as for the periodic form (the rule is built from the
    periodic functions; the imaginary-part copies test the same functions),
    and on the oracle's rule the matrices match the oracle's."""
    base = W.small("lih", mesh=(2, 2, 3), fe_order=2, a=4.8, re=1.6, rc=2.0)
    base["quad"] = {"n": 3, "n_ref": 6, "levels": 3, "mode": "error", "dist": 0.0, "tol": 1e-6}
    prob = B(base)
    say("bloch error rule")
    q = P.Problem(base).setup()
    p = P.Problem(prob).setup()
    for a, b in zip(P.pufe_get_leaves(p.ctx), P.pufe_get_leaves(q.ctx)):
        assert np.array_equal(a, b)
    q.close()
    o = oracle.Oracle(prob)
    lev, ijk, off = o.leaves()
    p.set_rule(lev, ijk, off)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    H, S = p.assemble(V, [KAP])
    Ho, So = o.assemble_dense_bloch(V.cpu().numpy(), KAP)
    eh, es = rel(p.to_dense(H[0]).cpu().numpy(), Ho), rel(p.to_dense(S[0]).cpu().numpy(), So)
    say("bloch error rule H", eh, "S", es)
    assert eh < TOL and es < TOL
    p.close()


@pytest.mark.parametrize("name", ["one-overlap-p1", "lih-p2"])
def test_bloch_nonlocal_term(name):
    """The separable nonlocal term over the Bloch-periodic basis: H against
    the oracle's H plus its nonlocal term at two k-points (the term alone to
    1e-9 of itself), S unchanged, FP64 and bf16x6 contractions."""
    prob = W.with_projectors(CASES[name][0]())
    say("bloch nonlocal", name)
    o, V = oracle_inputs(prob)
    p = P.Problem(prob).setup()
    Vd = torch.from_numpy(V).cuda()
    kpts = [KAP, (0.25, 0.25, -0.25)]
    H, S = p.assemble(Vd, kpts)
    H6, _ = p.assemble(Vd, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense_bloch(V, kap)
        Vn = o.nonlocal_dense(kap, bloch=True)
        Hg = p.to_dense(H[k]).cpu().numpy()
        eh, en = rel(Hg, Ho + Vn), rel(Hg - Ho, Vn)
        es = rel(p.to_dense(S[k]).cpu().numpy(), So)
        e6 = rel(p.to_dense(H6[k]).cpu().numpy(), Ho + Vn)
        say(name, kap, "H", eh, "term", en, "S", es, "bf16x6 H", e6, "|term|/|H|",
            np.linalg.norm(Vn) / np.linalg.norm(Ho))
        assert eh < TOL and en < 1e-9 and es < TOL and e6 < 1e-7
    p.close()
