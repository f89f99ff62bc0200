"""CPU tests of the C ABI: the library loads, exports what the header
declares, validates its inputs, and its host-side DOF map, enriched sets and
block layout agree with the oracle's.  No compute call is made."""
import copy
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

P = pytest.importorskip("paper_1611_00731_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "pufe.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(pufe_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(P.lib, n), n
    assert set(names) == set(P.EXPORTS)


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5):
        assert P.lib.pufe_error_string(code)
    assert P.lib.pufe_error_string(-99) == b"unknown error"


def _expect(code, fn):
    with pytest.raises(P.PufeError) as ei:
        fn()
    assert ei.value.code == code


def test_input_validation():
    base = W.small("one", mesh=(2, 2, 2), fe_order=1)
    ctx = P.pufe_create(0)
    try:
        _expect(-5, lambda: P.pufe_setup(ctx, stream=type("S", (), {"cuda_stream": 0})()))
        _expect(-5, lambda: P.pufe_query(ctx))
        _expect(-5, lambda: P.pufe_set_rule(ctx, [0], [[0, 0, 0]], [0, 1], stream=type("S", (), {"cuda_stream": 0})()))
        _expect(-1, lambda: P.pufe_set_problem(ctx, base["lattice"], [1, 2, 2], 1, base["atoms"],
                                               base["species"], base["enrichments"], base["quad"]))
        _expect(-1, lambda: P.pufe_set_problem(ctx, base["lattice"], [2, 2, 2], 4, base["atoms"],
                                               base["species"], base["enrichments"], base["quad"]))
        bad = [dict(base["enrichments"][0], l=4)]
        _expect(-1, lambda: P.pufe_set_problem(ctx, base["lattice"], [2, 2, 2], 1, base["atoms"],
                                               base["species"], bad, base["quad"]))
        bad = [dict(base["enrichments"][0], a=-1.0)]
        _expect(-1, lambda: P.pufe_set_problem(ctx, base["lattice"], [2, 2, 2], 1, base["atoms"],
                                               base["species"], bad, base["quad"]))
        lefty = np.diag([4.5, 4.5, -4.5])
        _expect(-1, lambda: P.pufe_set_problem(ctx, lefty, [2, 2, 2], 1, base["atoms"],
                                               base["species"], base["enrichments"], base["quad"]))
        skew = [[4.5, 0.2, 0.0], [0.0, 4.5, 0.0], [0.0, 0.0, 4.5]]
        q = dict(base["quad"], levels=1)
        _expect(-2, lambda: P.pufe_set_problem(ctx, skew, [2, 2, 2], 1, base["atoms"],
                                               base["species"], base["enrichments"], q))
        q = dict(base["quad"], n=13)
        _expect(-1, lambda: P.pufe_set_problem(ctx, base["lattice"], [2, 2, 2], 1, base["atoms"],
                                               base["species"], base["enrichments"], q))
        # a valid problem after rejected ones; assembly before setup is a state error
        P.pufe_set_problem(ctx, base["lattice"], [2, 2, 2], 1, base["atoms"], base["species"],
                           base["enrichments"], base["quad"])
        assert P.pufe_query(ctx)["n_elem"] == 8
        import ctypes as C
        k = (C.c_double * 3)(0, 0, 0)
        assert P.lib.pufe_assemble(ctx, None, k, 1, 0, 0, None, None, None) == -5
    finally:
        P.pufe_destroy(ctx)


PROBLEMS = {
    "single_atom_cube": W.single_atom_cube,
    "lih_cell": W.lih_cell,
    "ceal_cell": W.ceal_cell,
    "lih_supercell": W.lih_supercell,
    "lih-odd": lambda: W.small("lih", mesh=(3, 5, 3), fe_order=2, a=5.0),
    "one-p1": lambda: W.small("one", mesh=(2, 3, 4), fe_order=1, a=4.0),
    "ceal": lambda: W.small("ceal", mesh=(3, 3, 3), fe_order=2, a=5.0, rc=3.0, re=2.1),
    "skew": lambda: W.small("lih", mesh=(3, 2, 3), fe_order=2, levels=0,
                            lattice=[[5.0, 0.3, -0.2], [0.1, 4.8, 0.25], [0.2, -0.3, 5.3]]),
    "serendipity": lambda: W.small("lih", mesh=(3, 2, 4), fe_order=3, a=5.0),
    "serendipity-ceal": lambda: W.small("ceal", mesh=(2, 3, 2), fe_order=3, a=4.4, rc=3.0, re=2.4),
    "random-1": lambda: W.random_small(1),
    "random-7": lambda: W.random_small(7),
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_dof_map_and_enriched_sets_match_oracle(name):
    prob = PROBLEMS[name]()
    o = oracle.Oracle(prob)
    p = P.Problem(prob)
    try:
        lay = p.layout()
        assert np.array_equal(lay["dof_offset"], o.dof_offset())
        assert p.sizes["n_dof"] == o.n_dof
        assert p.sizes["n_fe_slots"] == o.n_fe_slots
    finally:
        p.close()


@pytest.mark.parametrize("name", ["single_atom_cube", "lih-odd", "one-p1", "ceal", "skew", "serendipity",
                                  "serendipity-ceal"])
def test_block_pattern_matches_element_coupling(name):
    prob = PROBLEMS[name]()
    o = oracle.Oracle(prob)
    p = P.Problem(prob)
    try:
        lay = p.layout()
        off = lay["dof_offset"]
        want = set()
        for e in range(o.n_elem):
            g, _ = o.element_dofs(e)
            v = np.searchsorted(off, g, side="right") - 1
            for a in set(v.tolist()):
                for b in set(v.tolist()):
                    want.add((a, b))
        got = set()
        rp, bc = lay["brow_ptr"], lay["bcol"]
        for v in range(len(rp) - 1):
            for k in range(rp[v], rp[v + 1]):
                got.add((v, int(bc[k])))
        assert got == want
        bo = lay["bval_offset"]
        sizes = np.diff(off)
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        assert np.array_equal(np.diff(bo), sizes[rows] * sizes[bc])
        assert bo[-1] == p.sizes["nnz"]
    finally:
        p.close()


def test_workload_sizes():
    """Sizes of the measured workloads (DOFs, BSR entries) from the host plan."""
    p = P.Problem(W.lih_cell())
    try:
        s = p.sizes
        assert (s["n_elem"], s["n_dof"], s["n_colors"]) == (512, 4888, 8)
        assert s["nnz"] == 1278838
    finally:
        p.close()


def test_golden_lih_cell_eigenvalues_file():
    """The stored oracle eigenvalues of the LiH-like cell (read by the GPU
    eigenvalue test and the benchmark): one per wanted eigenpair, finite and
    ascending."""
    import os
    import numpy as np
    import workloads as W
    ev = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "lih_cell_eigenvalues.txt"), comments="#")
    assert len(ev) == W.lih_cell()["n_eig"]
    assert np.all(np.diff(ev) >= 0)
    assert np.all(np.isfinite(ev))


@pytest.mark.parametrize("kind,mesh,p,a", [("lih", (2, 3, 2), 2, 4.6), ("one", (3, 3, 2), 1, 4.6),
                                            ("ceal", (2, 2, 2), 2, 4.6), ("ceal", (6, 5, 6), 1, 8.0),
                                            ("one", (6, 6, 5), 1, 8.0)])
def test_projector_pattern_holds_the_nonlocal_term(kind, mesh, p, a):
    """With projectors the BSR pattern also couples every pair of DOFs that
    reach one projector function, i.e. any image of its atom: every nonzero
    of the oracle's dense nonlocal term (eq. disceig3d) lies in a stored
    block, and the element-coupling blocks are all still there.  In the
    larger cells an atom next to a face or corner is reached through
    different images by vertices on opposite sides of the cell."""
    prob = W.with_projectors(W.small(kind, mesh=mesh, fe_order=p, levels=0, n=3, a=a))
    ctx = P.pufe_create(0)
    try:
        P.pufe_set_problem(ctx, prob["lattice"], prob["mesh"], prob["fe_order"], prob["atoms"],
                           prob["species"], prob["enrichments"], prob["quad"])
        lay0 = P.pufe_get_layout(ctx)
        P.pufe_set_projectors(ctx, prob["projectors"])
        lay = P.pufe_get_layout(ctx)
    finally:
        P.pufe_destroy(ctx)
    off = lay["dof_offset"]
    N = off[-1]
    stored = np.zeros((N, N), bool)
    for v in range(len(off) - 1):
        for k in range(lay["brow_ptr"][v], lay["brow_ptr"][v + 1]):
            w = lay["bcol"][k]
            stored[off[v]:off[v + 1], off[w]:off[w + 1]] = True
    for v in range(len(off) - 1):
        cols0 = set(lay0["bcol"][lay0["brow_ptr"][v]:lay0["brow_ptr"][v + 1]])
        assert cols0 <= set(lay["bcol"][lay["brow_ptr"][v]:lay["brow_ptr"][v + 1]])
    o = oracle.Oracle(prob)
    Vn = o.nonlocal_dense((0.1, -0.2, 0.3))
    assert np.abs(Vn[~stored]).max(initial=0.0) == 0.0
    assert np.count_nonzero(Vn) > 0


def test_projector_input_validation():
    base = W.small("one", mesh=(2, 2, 2), fe_order=1)
    ctx = P.pufe_create(0)
    try:
        _expect(-5, lambda: P.pufe_set_projectors(ctx, [{"species": 0, "l": 0, "a": 1.0, "rc": 1.0, "h": 1.0}]))
        P.pufe_set_problem(ctx, base["lattice"], base["mesh"], base["fe_order"], base["atoms"], base["species"],
                           base["enrichments"], base["quad"])
        _expect(-1, lambda: P.pufe_set_projectors(ctx, [{"species": 0, "l": 4, "a": 1.0, "rc": 1.0, "h": 1.0}]))
        _expect(-1, lambda: P.pufe_set_projectors(ctx, [{"species": 0, "l": 1, "a": -1.0, "rc": 1.0, "h": 1.0}]))
        P.pufe_set_projectors(ctx, [{"species": 0, "l": 1, "a": 1.0, "rc": 1.0, "h": 1.0}])
        P.pufe_set_projectors(ctx, [])
    finally:
        P.pufe_destroy(ctx)


def test_tabulated_radial_validation_and_layout():
    """Tabulated radials (section "Partition of unity enrichment functions")
    need 4..4096 finite samples and a known kind; they change the functions,
    not the enriched sets, so the layout equals the analytic problem's."""
    base = W.small("lih", mesh=(2, 3, 2), fe_order=2)
    tab = W.with_tabulated_radials(base, 12)

    def setp(ctx, prob):
        P.pufe_set_problem(ctx, prob["lattice"], prob["mesh"], prob["fe_order"], prob["atoms"], prob["species"],
                           prob["enrichments"], prob["quad"])

    ctx = P.pufe_create(0)
    try:
        setp(ctx, base)
        lay0 = P.pufe_get_layout(ctx)
        setp(ctx, tab)
        lay1 = P.pufe_get_layout(ctx)
        for k in lay0:
            assert np.array_equal(np.asarray(lay0[k]), np.asarray(lay1[k])), k
        bad = copy.deepcopy(tab)
        bad["enrichments"][0]["radial"] = [1.0, 0.5, 0.2]
        _expect(-1, lambda: setp(ctx, bad))
        bad = copy.deepcopy(tab)
        bad["enrichments"][1]["radial"][3] = float("nan")
        _expect(-1, lambda: setp(ctx, bad))
        bad = copy.deepcopy(tab)
        bad["enrichments"][0]["radial_kind"] = 2
        _expect(-1, lambda: setp(ctx, bad))
        setp(ctx, tab)   # still accepted after the refusals
    finally:
        P.pufe_destroy(ctx)


def test_enrichment_phase_validation_and_layout():
    """The Bloch-periodic enrichment (eq. Psi with f(R) = exp(i k.R)) keeps
    the DOFs and the block layout of the periodic form (with projectors too);
    the form is set after the problem and before set-up, and refuses elements
    whose real and imaginary rows exceed the kernels' function limit."""
    base = W.small("lih", mesh=(2, 3, 2), fe_order=2)

    def setp(ctx, prob):
        P.pufe_set_problem(ctx, prob["lattice"], prob["mesh"], prob["fe_order"], prob["atoms"], prob["species"],
                           prob["enrichments"], prob["quad"])

    ctx = P.pufe_create(0)
    try:
        _expect(-5, lambda: P.pufe_set_enrichment_phase(ctx, "bloch"))
        setp(ctx, base)
        lay0 = P.pufe_get_layout(ctx)
        P.pufe_set_enrichment_phase(ctx, "bloch")
        lay1 = P.pufe_get_layout(ctx)
        for k in lay0:
            assert np.array_equal(np.asarray(lay0[k]), np.asarray(lay1[k])), k
        assert P.pufe_query(ctx)["n_dof"] == oracle.Oracle(base).n_dof
        _expect(-1, lambda: P._check(ctx, P.lib.pufe_set_enrichment_phase(ctx, 2)))
        P.pufe_set_projectors(ctx, W.with_projectors(base)["projectors"])
        lay2 = P.pufe_get_layout(ctx)
        P.pufe_set_enrichment_phase(ctx, "periodic")
        lay3 = P.pufe_get_layout(ctx)
        for k in lay2:
            assert np.array_equal(np.asarray(lay2[k]), np.asarray(lay3[k])), k
        P.pufe_set_projectors(ctx, [])
        P.pufe_set_enrichment_phase(ctx, "bloch")
        ceal = W.small("ceal", mesh=(2, 2, 2), fe_order=1, rc=3.0, re=2.4)
        setp(ctx, ceal)
        _expect(-2, lambda: P.pufe_set_enrichment_phase(ctx, "bloch"))
    finally:
        P.pufe_destroy(ctx)


def test_element_function_limits():
    """64 enrichment functions on an element are accepted and 65 refused; with
    the Bloch-periodic enrichment 32 are accepted and 33 refused (their
    imaginary parts double them)."""
    def try_plan(prob, bloch=False):
        ctx = P.pufe_create(0)
        try:
            P.pufe_set_problem(ctx, prob["lattice"], prob["mesh"], prob["fe_order"], prob["atoms"],
                               prob["species"], prob["enrichments"], prob["quad"])
            if bloch:
                P.pufe_set_enrichment_phase(ctx, "bloch")
            return P.pufe_query(ctx)["max_nloc"]
        finally:
            P.pufe_destroy(ctx)

    assert try_plan(W.limit_cell(2)) == 8 + 64
    _expect(-2, lambda: try_plan(W.limit_cell(2, extra_h=True)))
    assert try_plan(W.limit_cell(1), bloch=True) == 8 + 64
    _expect(-2, lambda: try_plan(W.limit_cell(1, extra_h=True), bloch=True))
    assert oracle.Oracle(W.limit_cell(2)).element_dofs(0)[0].size == 8 + 64
    # 24 groups of mixed l on every element (44 functions on each of two vertices)
    assert try_plan(W.many_groups_cell()) == 8 + 88
    assert oracle.Oracle(W.many_groups_cell()).element_dofs(0)[0].size == 8 + 88
