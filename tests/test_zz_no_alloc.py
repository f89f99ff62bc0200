"""The allocation-free assembly entry (pufe_assemble_noalloc) against
pufe_assemble through the C ABI: two calls in a row on one GPU, the second
on a smaller problem, each compared with the allocating entry and with the
oracle; the fixed workspace's size limit gives a clear error."""
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


def _check(prob, kpts):
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    nnz = p.sizes["nnz"]
    for prec in ("fp64", "bf16x6"):
        Ha = torch.empty((len(kpts), nnz, 2), dtype=torch.float64, device="cuda")
        Sa = torch.empty_like(Ha)
        P.pufe_assemble(p.ctx, V, kpts, prec, "c128", Ha, Sa)
        Hn = torch.full_like(Ha, float("nan"))
        Sn = torch.full_like(Sa, float("nan"))
        P.pufe_assemble_noalloc(p.ctx, V, kpts, prec, "c128", Hn, Sn)
        torch.cuda.synchronize()
        # the same kernels in the same order: bitwise the allocating entry's result
        assert torch.equal(Hn, Ha) and torch.equal(Sn, Sa), prec
        k = len(kpts) - 1
        Ho, So = o.assemble_dense(V.cpu().numpy(), kpts[k])
        tol = 1e-12 if prec == "fp64" else 1e-7
        assert rel(p.to_dense(Hn[k]).cpu().numpy(), Ho) < tol
        assert rel(p.to_dense(Sn[k]).cpu().numpy(), So) < tol
    p.close()


def test_noalloc_matches_assemble_twice_then_smaller():
    big = W.small("lih", mesh=(3, 2, 2), fe_order=2, levels=1, n=3, a=5.0)
    small = W.small("lih", mesh=(2, 2, 2), fe_order=1, levels=1, n=2, a=4.6)
    say("noalloc: larger problem, 3 k-points")
    _check(big, [(0.0, 0.0, 0.0), (0.12, -0.24, 0.37), (0.25, 0.25, -0.25)])
    say("noalloc: smaller problem, 2 k-points")
    _check(small, [(0.0, 0.0, 0.0), (0.31, 0.0, -0.2)])


def test_noalloc_rejects_a_problem_beyond_the_workspace():
    prob = W.lih_cell()   # K-chunk partial tiles of about 190 MB
    say("noalloc: size limit")
    p = P.Problem(prob).setup()
    V = torch.zeros(p.sizes["n_qp"], dtype=torch.float64, device="cuda")
    H = torch.zeros((1, p.sizes["nnz"], 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PufeError) as err:
        P.pufe_assemble_noalloc(p.ctx, V, [(0.0, 0.0, 0.0)], "fp64", "c128", H, None)
    assert err.value.code == -2 and "workspace" in str(err.value)
    torch.cuda.synchronize()
    assert bool((H == 0).all())   # nothing was launched
    p.close()
