"""GPU parity of the separable nonlocal term (eq. disceig3d) against the
oracle, through the C ABI: H of the library equals the oracle's H plus its
dense nonlocal term sum_J h_J f_J^i conj(f_J^j) at Gamma and general
k-points, for trilinear and triquadratic meshes, elements of many functions
(several row blocks of projector coefficients), refined elements (several
K-chunks), a skewed triclinic cell on the oracle's own error-driven rule, and
every output type; S is unchanged.  FP64 to 1e-12; the bf16x6 contraction
(the nonlocal term stays FP64) to 1e-7."""
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


CASES = {
    "lih-p2": (lambda: W.with_projectors(W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)),
               [(0.0, 0.0, 0.0), (0.12, -0.24, 0.37), (0.25, 0.25, -0.25)]),
    "one-p1": (lambda: W.with_projectors(W.small("one", mesh=(3, 3, 2), fe_order=1, levels=2, n=3, a=4.6)),
               [(0.31, 0.0, -0.2)]),
    "ceal-many": (lambda: W.with_projectors(W.small("ceal", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4,
                                                    rc=3.0, re=2.4)), [(0.0, 0.0, 0.0), (0.25, -0.25, 0.25)]),
    "ceal-triclinic": (lambda: W.with_projectors(W.ceal_triclinic(mesh=3, levels=1, n=3, n_ref=5, tol=1e-4)),
                       W.PAPER_KPTS),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_nonlocal_assembly_matches_oracle(name):
    make, kpts = CASES[name]
    prob = make()
    say("nonlocal", name)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    if prob["quad"]["mode"] == "error":   # assemble on the oracle's rule
        lev, ijk, loff = o.leaves()
        p.set_rule(lev, ijk, loff)
    Vh = V.cpu().numpy()
    H, S = p.assemble(V, kpts)
    Hs, _ = p.assemble(V, kpts, precision="bf16x6")
    for k, kap in enumerate(kpts):
        Ho, So = o.assemble_dense(Vh, kap)
        Vn = o.nonlocal_dense(kap)
        Hg = p.to_dense(H[k]).cpu().numpy()
        eh = rel(Hg, Ho + Vn)
        es = rel(p.to_dense(S[k]).cpu().numpy(), So)
        e6 = rel(p.to_dense(Hs[k]).cpu().numpy(), Ho + Vn)
        # the nonlocal part on its own: what the library added beyond the
        # local H, against the oracle's term (the local part's rounding,
        # ~1e-15 of |H|, is far below it)
        en = rel(Hg - Ho, Vn)
        say(name, kap, "H", eh, "S", es, "bf16x6 H", e6, "nonlocal part", en, "|Vnl|/|H|",
            np.abs(Vn).max() / np.abs(Ho).max())
        assert eh < 1e-12 and es < 1e-12 and e6 < 1e-7 and en < 1e-9
    p.close()


def test_nonlocal_output_types_and_refusals():
    """Real Gamma and complex64 outputs carry the term too; the allocation-free
    entry and the batch refuse problems with projectors."""
    prob = W.with_projectors(W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0))
    say("nonlocal output types")
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    Ho, So = o.assemble_dense(V.cpu().numpy())
    ref = (Ho + o.nonlocal_dense()).real
    Hr, _ = p.assemble(V, [(0.0, 0.0, 0.0)], out_dtype="f64")
    assert rel(p.to_dense(Hr[0], "f64").real.cpu().numpy(), ref) < 1e-12
    kap = (0.12, -0.24, 0.37)
    H32, _ = p.assemble(V, [kap], out_dtype="c64")
    Hc = H32[0].double().contiguous()
    ref = o.assemble_dense(V.cpu().numpy(), kap)[0] + o.nonlocal_dense(kap)
    assert rel(p.to_dense(Hc).cpu().numpy(), ref) < 1e-6
    H = torch.empty((1, p.sizes["nnz"], 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PufeError) as err:
        P.pufe_assemble_noalloc(p.ctx, V, [kap], "fp64", "c128", H, None)
    assert err.value.code == -2
    with pytest.raises(P.PufeError):
        P.Batch([p])
    p.close()


def _golden_projector_coefficients():
    """Sample functions, h_J and, per k-point, the oracle's f_J^i on the
    sample (tests/golden/lih_cell_projector_coefficients.txt, written by
    make_lih_cell_projector_coefficients.py from the oracle alone)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "lih_cell_projector_coefficients.txt")
    lines = [ln.split() for ln in open(path) if not ln.startswith("#")]
    idx = np.array(lines[0][1:], np.int64)
    h = np.array(lines[1][1:], float)
    ks, Fs, i = [], [], 2
    while i < len(lines):
        ks.append(tuple(map(float, lines[i][1:])))
        rows = np.array([list(map(float, r)) for r in lines[i + 1:i + 1 + len(h)]])
        Fs.append(rows[:, 0::2] + 1j * rows[:, 1::2])
        i += 1 + len(h)
    return idx, h, ks, Fs


def test_lih_cell_full_size_nonlocal_term():
    """The LiH-like cell at full size (512 elements, 1.52 M points, N = 4888)
    with its Li s+p and H s projectors: on a sample of 66 functions (those
    of the vertices next to a Li and an H atom and seeded random ones), the
    difference between the library's H with and without projectors equals
    the stored oracle term sum_J h_J f_J^i conj(f_J^j), at Gamma and a
    general k-point; S is bitwise unchanged."""
    idx, h, kpts, Fs = _golden_projector_coefficients()
    say("nonlocal lih_cell full size", len(idx), "sampled functions")
    out = {}
    for tag, prob in (("local", W.lih_cell()), ("nonlocal", W.with_projectors(W.lih_cell()))):
        p = P.Problem(prob).setup()
        xyz, _, _ = p.quadrature()
        V = potential_at(xyz, prob)
        del xyz
        H, S = p.assemble(V, kpts)
        sel = torch.from_numpy(idx).cuda()
        out[tag] = [(p.to_dense(H[k])[sel][:, sel].cpu().numpy(), p.to_dense(S[k])[sel][:, sel].cpu().numpy())
                    for k in range(len(kpts))]
        del H, S, V
        p.close()
    for k, kap in enumerate(kpts):
        F = Fs[k]
        ref = (F * h[:, None]).T @ F.conj()     # [i][j] = sum_J h_J f_J^i conj(f_J^j)
        diff = out["nonlocal"][k][0] - out["local"][k][0]
        e = rel(diff, ref)
        say("lih_cell", kap, "nonlocal term on the sample", e, "max |term|", np.abs(ref).max(),
            "coupled pairs", int((np.abs(ref) > 0).sum()))
        assert np.abs(ref).max() > 1e-4 and e < 1e-9
        assert np.array_equal(out["nonlocal"][k][1], out["local"][k][1])
