"""Problems at the kernels' per-element limits against the oracle: elements
reached by exactly 64 enrichment functions in 16 groups (the most an element
may hold), and, with the Bloch-periodic enrichment, by exactly 32 (whose
imaginary parts double them to 64).  One function more is refused on the host
(tests/test_abi_cpu.py).  Elements of 24 groups of mixed l (17, 5, 1, 1 of
l = 0 .. 3) in the wide work groups, whose enrichment schedule then packs the
groups instead of giving each l waves of its own."""
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


@pytest.mark.parametrize("form", ["periodic", "bloch"])
def test_element_function_limit(form):
    prob = W.limit_cell(2 if form == "periodic" else 1)
    if form == "bloch":
        prob = W.with_bloch_enrichment(prob)
    say("function limit", form)
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    kap = (0.15, -0.3, 0.2)
    H, S = p.assemble(V, [kap])
    H6, S6 = p.assemble(V, [kap], precision="bf16x6")
    Vh = V.cpu().numpy()
    Ho, So = o.assemble_dense_bloch(Vh, kap) if form == "bloch" else o.assemble_dense(Vh, kap)
    eh, es = rel(p.to_dense(H[0]).cpu().numpy(), Ho), rel(p.to_dense(S[0]).cpu().numpy(), So)
    e6 = max(rel(p.to_dense(H6[0]).cpu().numpy(), Ho), rel(p.to_dense(S6[0]).cpu().numpy(), So))
    say(form, "rows", p.sizes["max_nloc"], "H", eh, "S", es, "bf16x6", e6)
    assert eh < 1e-12 and es < 1e-12 and e6 < 1e-7
    p.close()


def test_many_groups_of_mixed_l():
    prob = W.many_groups_cell()
    say("many groups")
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = potential_at(torch.from_numpy(xyz).cuda(), prob)
    p = P.Problem(prob).setup()
    assert p.sizes["max_nloc"] == 96   # six tiles: the wide kernel
    kap = (0.15, -0.3, 0.2)
    H, S = p.assemble(V, [kap])
    H6, S6 = p.assemble(V, [kap], precision="bf16x6")
    Ho, So = o.assemble_dense(V.cpu().numpy(), kap)
    eh, es = rel(p.to_dense(H[0]).cpu().numpy(), Ho), rel(p.to_dense(S[0]).cpu().numpy(), So)
    e6 = max(rel(p.to_dense(H6[0]).cpu().numpy(), Ho), rel(p.to_dense(S6[0]).cpu().numpy(), So))
    say("many groups H", eh, "S", es, "bf16x6", e6)
    assert eh < 1e-12 and es < 1e-12 and e6 < 1e-7
    p.close()
