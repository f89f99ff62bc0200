"""The persistent, graph-captured batch over lattice constants and k-points
against the oracle, and graph replays against each other."""
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


def test_batch_small_sweep_vs_oracle():
    base = W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0)
    probs = [W.with_lattice_constant(base, a) for a in (4.6, 5.0, 5.4)]
    kpts = W.mp2()[:3]
    say("batch small sweep")
    oracles, Vs, ps = [], [], []
    for pr in probs:
        o = oracle.Oracle(pr)
        xyz, _, _ = o.quadrature()
        oracles.append(o)
        Vs.append(potential_at(torch.from_numpy(xyz).cuda(), pr))
        ps.append(P.Problem(pr).setup())
    b = P.Batch(ps)
    Hs, Ss = b.alloc(len(kpts), device="cuda")
    b.assemble(Vs, kpts, Hs, Ss)
    torch.cuda.synchronize()
    for i, (o, p) in enumerate(zip(oracles, ps)):
        for k, kap in enumerate(kpts):
            Ho, So = o.assemble_dense(Vs[i].cpu().numpy(), kap)
            assert rel(p.to_dense(Hs[i][k]).cpu().numpy(), Ho) < 1e-12
            assert rel(p.to_dense(Ss[i][k]).cpu().numpy(), So) < 1e-12
    # replays with eager work in between stay identical
    ref = [h.clone() for h in Hs]
    for _ in range(3):
        for h in Hs:
            h.fill_(7.0)
        torch.cuda.synchronize()
        b.assemble(Vs, kpts, Hs, Ss)
        torch.cuda.synchronize()
        for h, r in zip(Hs, ref):
            assert torch.equal(h, r)
    # split precision through the same batch
    b.assemble(Vs, kpts, Hs, Ss, precision="bf16x6")
    torch.cuda.synchronize()
    Ho, So = oracles[1].assemble_dense(Vs[1].cpu().numpy(), kpts[2])
    assert rel(ps[1].to_dense(Hs[1][2]).cpu().numpy(), Ho) < 1e-7
    b.close()
    for p in ps:
        p.close()


def test_batch_general_variant_problems_vs_oracle():
    """A batch of problems that need the general kernel variants (cubic
    serendipity elements, tabulated radials, wide elements) next to an
    analytic/Lagrange one: every output against the oracle, FP64 and bf16x6."""
    probs = [W.small("one", mesh=(2, 3, 2), fe_order=3, levels=1, n=3, a=4.6),
             W.with_tabulated_radials(W.small("lih", mesh=(3, 2, 2), fe_order=1, levels=1, n=3, a=5.0), 40),
             W.small("ceal", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4, rc=3.0, re=2.4)]
    kpts = W.mp2()[:2]
    say("batch general-variant problems")
    oracles, Vs, ps = [], [], []
    for pr in probs:
        o = oracle.Oracle(pr)
        xyz, _, _ = o.quadrature()
        oracles.append(o)
        Vs.append(potential_at(torch.from_numpy(xyz).cuda(), pr))
        ps.append(P.Problem(pr).setup())
    b = P.Batch(ps)
    for prec, tol in (("fp64", 1e-12), ("bf16x6", 1e-7)):
        Hs, Ss = b.alloc(len(kpts), device="cuda")
        b.assemble(Vs, kpts, Hs, Ss, precision=prec)
        torch.cuda.synchronize()
        for i, (o, p) in enumerate(zip(oracles, ps)):
            for k, kap in enumerate(kpts):
                Ho, So = o.assemble_dense(Vs[i].cpu().numpy(), kap)
                eh = rel(p.to_dense(Hs[i][k]).cpu().numpy(), Ho)
                es = rel(p.to_dense(Ss[i][k]).cpu().numpy(), So)
                say(prec, probs[i]["name"], kap, "H", eh, "S", es)
                assert eh < tol and es < tol
    b.close()
    for p in ps:
        p.close()


def test_batch_lih_lattice_sweep_full_size_sampled():
    """The 11 lattice constants x 8 k-points sweep (88 assemblies in one
    persistent launch): sampled BSR blocks against the oracle."""
    probs = W.lih_lattice_sweep()
    kpts = W.mp2()
    say("batch lih_lattice_sweep full size")
    ps, Vs, oracles, Vh = [], [], [], []
    for pr in probs:
        o = oracle.Oracle(pr)
        xyz, _, _ = o.quadrature()
        V = potential_at(torch.from_numpy(xyz).cuda(), pr)
        oracles.append(o)
        Vs.append(V)
        Vh.append(V.cpu().numpy())
        ps.append(P.Problem(pr).setup())
    b = P.Batch(ps)
    Hs, Ss = b.alloc(len(kpts), device="cuda")
    b.assemble(Vs, kpts, Hs, Ss)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for i in (0, 5, 10):
        lay = ps[i].layout()
        off = lay["dof_offset"]
        for k in (0, 3, 7):
            v = int(rng.integers(0, len(off) - 1))
            kk = int(rng.integers(lay["brow_ptr"][v], lay["brow_ptr"][v + 1]))
            w = int(lay["bcol"][kk])
            Hb, Sb = oracles[i].assemble_block(Vh[i], kpts[k], v, w)
            b0, b1 = lay["bval_offset"][kk], lay["bval_offset"][kk + 1]
            shape = (off[v + 1] - off[v], off[w + 1] - off[w])
            Hg = Hs[i][k, b0:b1].cpu().numpy()
            Sg = Ss[i][k, b0:b1].cpu().numpy()
            assert rel((Hg[:, 0] + 1j * Hg[:, 1]).reshape(shape), Hb) < 1e-12
            assert rel((Sg[:, 0] + 1j * Sg[:, 1]).reshape(shape), Sb) < 1e-12
    b.close()
    for p in ps:
        p.close()


def test_autotuner_cache_and_parity(tmp_path):
    prob = W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)
    say("autotuner")
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    cache = tmp_path / "tune.json"
    p = P.Problem(prob).setup()
    P.pufe_tune(p.ctx, "fp64", str(cache))
    import json
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (k, v), = entries.items()
    assert "gfx950" in k and v["block"] in (2, 3, 4) and v["items"] > 0
    kap = (0.12, -0.24, 0.37)
    H, S = p.assemble(V, [kap])
    Ho, So = o.assemble_dense(V.cpu().numpy(), kap)
    assert rel(p.to_dense(H[0]).cpu().numpy(), Ho) < 1e-12
    # a second context reads the cached choice
    p2 = P.Problem(prob).setup()
    P.pufe_tune(p2.ctx, "fp64", str(cache))
    assert json.loads(cache.read_text()) == entries
    H2, _ = p2.assemble(V, [kap])
    assert torch.equal(H2, H)
    p.close()
    p2.close()


def test_batch_refuses_a_context_tuned_after_creation():
    """A batch copies the work items of the plans it was created on; tuning a
    context afterwards re-plans it, so the batch must refuse to run (before
    launching anything) instead of reading freed tables, and a batch created
    anew runs and matches the oracle."""
    base = W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0)
    probs = [W.with_lattice_constant(base, a) for a in (4.8, 5.2)]
    kpts = W.mp2()[:2]
    say("batch after tune")
    ps, Vs, oracles = [], [], []
    for pr in probs:
        o = oracle.Oracle(pr)
        xyz, _, _ = o.quadrature()
        oracles.append(o)
        Vs.append(potential_at(torch.from_numpy(xyz).cuda(), pr))
        ps.append(P.Problem(pr).setup())
    b = P.Batch(ps)
    Hs, Ss = b.alloc(len(kpts), device="cuda")
    b.assemble(Vs, kpts, Hs, Ss)
    torch.cuda.synchronize()
    P.pufe_tune(ps[1].ctx, "fp64", None)
    for h in Hs:
        h.fill_(3.0)
    with pytest.raises(P.PufeError) as err:
        b.assemble(Vs, kpts, Hs, Ss)
    assert err.value.code == -5   # PUFE_ERR_STATE
    torch.cuda.synchronize()
    assert all(bool((h == 3.0).all()) for h in Hs)   # nothing was launched
    b.close()
    b2 = P.Batch(ps)
    b2.assemble(Vs, kpts, Hs, Ss)
    torch.cuda.synchronize()
    for i, (o, p) in enumerate(zip(oracles, ps)):
        Ho, So = o.assemble_dense(Vs[i].cpu().numpy(), kpts[1])
        assert rel(p.to_dense(Hs[i][1]).cpu().numpy(), Ho) < 1e-12
        assert rel(p.to_dense(Ss[i][1]).cpu().numpy(), So) < 1e-12
    b2.close()
    for p in ps:
        p.close()


def test_batch_tuned_stage_lengths_c64_and_split(tmp_path):
    """Problems whose cached tuner choices give them different stage lengths
    (32, 16 and 24 points per stage) run in one batch, each length in a
    persistent launch of its own: FP64 with complex128 and complex64 outputs
    and bf16x6 with complex64 outputs against the oracle, on three k-points."""
    import json
    probs = [W.small("lih", mesh=(2, 3, 2), fe_order=2, levels=1, n=3, a=5.0),
             W.small("lih", mesh=(3, 3, 2), fe_order=2, levels=1, n=3, a=5.2),
             W.small("ceal", mesh=(2, 2, 2), fe_order=2, levels=1, n=3, a=4.4)]
    kpts = W.mp2()[:3]
    say("batch tuned stage lengths, c64, bf16x6")
    cache = tmp_path / "tune.json"
    for pr in probs:
        p = P.Problem(pr).setup()
        P.pufe_tune(p.ctx, "fp64", str(cache))
        p.close()
    entries = json.loads(cache.read_text())
    assert len(entries) == 3
    for v, q in zip(entries.values(), (32, 16, 24)):
        v["q"] = q
    cache.write_text(json.dumps(entries))   # compact separators: the form the library parses
    ps, Vs, oracles = [], [], []
    for pr in probs:
        o = oracle.Oracle(pr)
        xyz, _, _ = o.quadrature()
        oracles.append(o)
        Vs.append(potential_at(torch.from_numpy(xyz).cuda(), pr))
        p = P.Problem(pr).setup()
        P.pufe_tune(p.ctx, "fp64", str(cache))   # applies the cached choice
        ps.append(p)
    assert json.loads(cache.read_text()) == entries
    b = P.Batch(ps)
    refs = [[o.assemble_dense(Vs[i].cpu().numpy(), kap) for kap in kpts] for i, o in enumerate(oracles)]
    for prec, dt, tol in (("fp64", "c128", 1e-12), ("fp64", "c64", 1e-6), ("bf16x6", "c64", 1e-6)):
        Hs, Ss = b.alloc(len(kpts), out_dtype=dt, device="cuda")
        b.assemble(Vs, kpts, Hs, Ss, precision=prec, out_dtype=dt)
        torch.cuda.synchronize()
        worst = 0.0
        for i, p in enumerate(ps):
            for k in range(len(kpts)):
                Ho, So = refs[i][k]
                worst = max(worst, rel(p.to_dense(Hs[i][k].double().contiguous()).cpu().numpy(), Ho),
                            rel(p.to_dense(Ss[i][k].double().contiguous()).cpu().numpy(), So))
        say(prec, dt, "worst relative error", worst)
        assert worst < tol
    b.close()
    for p in ps:
        p.close()
