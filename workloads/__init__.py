"""Seeded synthetic inputs for the PUFE assembly path.

This module only *describes* problems (cells, meshes, atoms, enrichment
descriptors, quadrature parameters, k-points) and draws the random numbers the
workloads need (atomic jitter, adjoint factors).  It holds none of the
method's arithmetic: no basis functions, quadrature rules or matrix elements.
Both the HIP library (through its Python binding) and the CPU oracle consume
the dictionaries built here.

Problem dictionary keys
-----------------------
lattice      3x3 nested list, rows a_1, a_2, a_3 (bohr), right-handed.
mesh         [n1, n2, n3] hexahedral elements along a_1, a_2, a_3.
fe_order     1 (8-node trilinear), 2 (27-node triquadratic Lagrange) or 3
             (32-node cubic serendipity).
atoms        list of Cartesian positions [x, y, z] (bohr).
species      list of species indices, one per atom.
species_info list of {"name", "Z", "rloc"} (used only by the potential).
enrichments  list of {"species", "l", "a", "rc", "re"}: each descriptor adds
             the 2l+1 functions r^l exp(-a r^2) (1-(r/rc)^2)^3 Y_lm around
             every atom of that species, on every vertex closer than re.
             An optional "radial" (list of n >= 4 samples of the pseudoatomic
             radial divided by r^l at r_j = j rc/(n-1)) replaces the analytic
             radial by r^l times the cubic spline through the samples times
             the C^3 cutoff.
quad         {"n", "n_ref", "levels", "mode" ("geom"|"error"), "dist", "tol"}.
kpts         list of reduced k-points kappa (k = sum kappa_i b_i).
n_eig        number of lowest eigenpairs wanted.
"""
from __future__ import annotations

import copy
import math

import numpy as np

__all__ = [
    "single_atom_cube", "lih_cell", "lih_lattice_sweep", "ceal_cell", "lih_supercell", "small", "lih_table1",
    "ceal_triclinic", "PAPER_KPTS", "with_projectors", "with_tabulated_radials",
    "mp2", "ceal_kpoints", "jitter", "adjoint_factor", "with_lattice_constant",
    "orthorhombic", "random_small",
]

MP2 = [[sx * 0.25, sy * 0.25, sz * 0.25]
       for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)]


def mp2():
    """Monkhorst-Pack 2x2x2 set in reduced coordinates: (+-1/4)^3, 8 points."""
    return copy.deepcopy(MP2)


def ceal_kpoints():
    """Time-reversal-reduced MP 2x2x2 set (4 points) for the CeAl-like cell."""
    return [[0.25, 0.25, 0.25], [0.25, 0.25, -0.25],
            [0.25, -0.25, 0.25], [-0.25, 0.25, 0.25]]


def jitter(n_atoms: int, sigma: float = 0.05, seed: int = 0) -> np.ndarray:
    """Gaussian displacements N(0, sigma) per coordinate (PCG64, given seed),
    drawn atom by atom in list order."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, size=(n_atoms, 3))


def adjoint_factor(n: int, rank: int = 128, seed: int = 0) -> np.ndarray:
    """C (n x rank) complex with entries CN(0, 1/n) from PCG64(seed).

    The adjoint matrix used by the backward tests is P = C C^H, evaluated only
    on the sparsity pattern of H.
    """
    rng = np.random.default_rng(seed)
    s = math.sqrt(0.5 / n)
    re = rng.normal(0.0, s, size=(n, rank))
    im = rng.normal(0.0, s, size=(n, rank))
    return re + 1j * im


def cubic(a: float):
    return [[a, 0.0, 0.0], [0.0, a, 0.0], [0.0, 0.0, a]]


def orthorhombic(lattice) -> bool:
    lat = np.asarray(lattice, float)
    return bool(np.all(lat - np.diag(np.diag(lat)) == 0.0))


def _problem(lattice, mesh, fe_order, atoms, species, species_info, enrichments,
             quad, kpts, n_eig, name):
    return {
        "name": name,
        "lattice": [list(map(float, r)) for r in lattice],
        "mesh": list(map(int, mesh)),
        "fe_order": int(fe_order),
        "atoms": [list(map(float, p)) for p in atoms],
        "species": list(map(int, species)),
        "species_info": species_info,
        "enrichments": enrichments,
        "quad": quad,
        "kpts": [list(map(float, k)) for k in kpts],
        "n_eig": int(n_eig),
        "potential": {"cutoff": 12.0},
    }


def single_atom_cube():
    """Single-atom cube: side 4.0, 4^3 trilinear, 5^3 Gauss, no refinement;
    s enrichment a=1.0, rc=2.5, support radius 1.5; Gamma; 4 eigenpairs."""
    return _problem(
        cubic(4.0), [4, 4, 4], 1, [[0.0, 0.0, 0.0]], [0],
        [{"name": "X", "Z": 1.0, "rloc": 0.5}],
        [{"species": 0, "l": 0, "a": 1.0, "rc": 2.5, "re": 1.5}],
        {"n": 5, "n_ref": 8, "levels": 0, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        [[0.0, 0.0, 0.0]], 4, "single_atom_cube")


LIH_ENR = [
    {"species": 0, "l": 0, "a": 2.0, "rc": 3.0, "re": 2.0},   # Li s
    {"species": 0, "l": 0, "a": 0.3, "rc": 3.0, "re": 2.0},   # Li s
    {"species": 0, "l": 1, "a": 0.5, "rc": 3.0, "re": 2.0},   # Li p
    {"species": 1, "l": 0, "a": 0.8, "rc": 3.0, "re": 2.0},   # H s
]
LIH_SPECIES = [{"name": "Li", "Z": 3.0, "rloc": 0.4},
               {"name": "H", "Z": 1.0, "rloc": 0.4}]
FCC = [(0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]


def _lih_reduced(cells=1):
    """Reduced positions and species of the rock-salt LiH cell (or a cells^3
    supercell of it), in the order Li0, H0, Li1, H1, ... per unit cell, unit
    cells in lexicographic order (x fastest)."""
    red, spc = [], []
    for t3 in range(cells):
        for t2 in range(cells):
            for t1 in range(cells):
                for f in FCC:
                    li = np.array([(f[0] + t1), (f[1] + t2), (f[2] + t3)]) / cells
                    h = li + np.array([0.5, 0.0, 0.0]) / cells
                    red += [li, h]
                    spc += [0, 1]
    return np.array(red), spc


def lih_cell(a: float = 7.6, mesh=8):
    """Rock-salt LiH-like cell (4 Li + 4 H), jittered N(0, 0.05) seed 0,
    triquadratic mesh^3, 6^3 Gauss + 2 geometric octree levels within 1 bohr."""
    red, spc = _lih_reduced(1)
    pos = red * a + jitter(len(spc))
    return _problem(
        cubic(a), [mesh] * 3, 2, pos, spc, LIH_SPECIES, copy.deepcopy(LIH_ENR),
        {"n": 6, "n_ref": 8, "levels": 2, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        [[0.0, 0.0, 0.0]], 16, "lih_cell")


def with_lattice_constant(prob, a: float):
    """Same problem at lattice constant a: the reduced lattice positions scale,
    the absolute jitter stays the same (the lattice-constant sweep)."""
    a0 = prob["lattice"][0][0]
    red, _ = _lih_reduced(1)
    jit = np.asarray(prob["atoms"]) - red * a0
    out = copy.deepcopy(prob)
    out["lattice"] = cubic(a)
    out["atoms"] = (red * a + jit).tolist()
    out["name"] = f"{prob['name']}@a={a:.2f}"
    return out


def lih_lattice_sweep():
    """The LiH-like cell at 11 lattice constants 6.80..8.40 with the 8-point
    MP 2x2x2 k set: a list of 11 problems (88 assemblies)."""
    base = lih_cell()
    out = []
    for i in range(11):
        a = round(6.8 + 0.16 * i, 10)
        p = with_lattice_constant(base, a)
        p["kpts"] = mp2()
        out.append(p)
    return out


def ceal_cell():
    """CsCl CeAl-like cell a=5.8: Ce at 0, Al at the body centre; 12^3
    triquadratic, 8^3 Gauss + 3 octree levels within 1 bohr; Ce s,p,d,f x
    {3.0, 0.4} (32 functions), Al s,p,d (0.6) (9 functions), rc = 4,
    support radius 2.5; 4 k-points."""
    a = 5.8
    enr = []
    for l in range(4):
        for ex in (3.0, 0.4):
            enr.append({"species": 0, "l": l, "a": ex, "rc": 4.0, "re": 2.5})
    for l in range(3):
        enr.append({"species": 1, "l": l, "a": 0.6, "rc": 4.0, "re": 2.5})
    return _problem(
        cubic(a), [12] * 3, 2, [[0.0, 0.0, 0.0], [a / 2, a / 2, a / 2]], [0, 1],
        [{"name": "Ce", "Z": 12.0, "rloc": 0.3}, {"name": "Al", "Z": 3.0, "rloc": 0.3}],
        enr,
        {"n": 8, "n_ref": 10, "levels": 3, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        ceal_kpoints(), 16, "ceal_cell")


# The two k-points of the paper's LiH and CeAl runs, read as reduced
# coordinates (section "Self-consistent calculations").
PAPER_KPTS = [[0.0, 0.0, 0.0], [0.12, -0.24, 0.37]]


def ceal_triclinic(mesh: int = 12, levels: int = 2, n: int = 6, n_ref: int = 8, tol: float = 1e-5):
    """The paper's triclinic CeAl cell (eq. ceal-primitive): primitive vectors
    a (1.00, 0.02, -0.04), a (0.01, 0.98, 0.03), a (0.03, -0.06, 1.09), a = 5.75
    bohr, Ce at (0.01, 0.02, 0.03) and Al at (0.51, 0.47, 0.55) in lattice
    coordinates; its two k-points.  Skewed element maps, so the rule is the
    paper's error-driven one (base n^3 against reference n_ref^3 Gauss on
    Psi^2 and |grad Psi|^2, absolute tolerance tol, up to `levels` levels).
    The enrichments, potential and radial functions are those of the
    CeAl-like cell (the paper's own need its pseudopotential tables)."""
    a = 5.75
    lat = a * np.array([[1.00, 0.02, -0.04], [0.01, 0.98, 0.03], [0.03, -0.06, 1.09]])
    red = np.array([[0.01, 0.02, 0.03], [0.51, 0.47, 0.55]])
    enr = []
    for l in range(4):
        for ex in (3.0, 0.4):
            enr.append({"species": 0, "l": l, "a": ex, "rc": 4.0, "re": 2.5})
    for l in range(3):
        enr.append({"species": 1, "l": l, "a": 0.6, "rc": 4.0, "re": 2.5})
    return _problem(
        lat, [mesh] * 3, 2, red @ lat, [0, 1],
        [{"name": "Ce", "Z": 12.0, "rloc": 0.3}, {"name": "Al", "Z": 3.0, "rloc": 0.3}],
        enr, {"n": n, "n_ref": n_ref, "levels": levels, "mode": "error", "dist": 0.0, "tol": tol},
        copy.deepcopy(PAPER_KPTS), 16, f"ceal_triclinic-{mesh}")


# Synthetic separable-projector sets (eq. disceig3d nonlocal term) in the
# radial form of the enrichments: per species name, (l, a, rc, h) rows.  They
# stand in for tabulated pseudopotential projectors (not available here).
PROJECTORS = {
    "Li": [(0, 1.5, 2.0, 0.8), (1, 1.2, 2.0, -0.3)],
    "H": [(0, 2.0, 1.5, 0.5)],
    "Ce": [(0, 2.5, 1.8, 1.1), (1, 2.0, 1.8, -0.4), (2, 1.8, 1.8, 0.3)],
    "Al": [(0, 1.6, 1.8, 0.6), (1, 1.4, 1.8, -0.2)],
    "X": [(0, 1.5, 1.6, 0.7), (1, 1.3, 1.6, -0.3)],
}


def with_projectors(prob, scale_rc: float = 1.0):
    """A copy of prob with the synthetic projector set of each of its species
    (cutoffs scaled by scale_rc)."""
    out = copy.deepcopy(prob)
    proj = []
    for sp, info in enumerate(prob["species_info"]):
        for l, a, rc, h in PROJECTORS[info["name"]]:
            proj.append({"species": sp, "l": l, "a": a, "rc": rc * scale_rc, "h": h})
    out["projectors"] = proj
    out["name"] = prob["name"] + "+nl"
    return out


def with_tabulated_radials(prob, n_samples: int = 48):
    """A copy of prob whose enrichment radials are given as tables, as a
    radial solver would output them: each descriptor gets "radial", the
    n_samples values of its pseudoatomic radial divided by r^l, here the
    Gaussian exp(-a r^2), at r_j = j rc / (n_samples - 1)."""
    out = copy.deepcopy(prob)
    for e in out["enrichments"]:
        r = np.linspace(0.0, e["rc"], n_samples)
        e["radial"] = np.exp(-e["a"] * r * r).tolist()
    out["name"] = prob["name"] + "+tab"
    return out


def limit_cell(n_ce: int = 2, extra_h: bool = False):
    """A 2^3 trilinear cube (a = 4.4, every element's corners are all 8
    vertices) with n_ce Ce-like atoms, each right next to its own vertex and
    carrying 32 functions (s, p, d, f x 2 exponents, rc = 3, re = 0.5), so
    every element is reached by 32 n_ce enrichment functions in 8 n_ce
    groups; extra_h adds an H-like atom with one s function next to a third
    vertex (one function over the limit when n_ce = 2)."""
    a = 4.4
    pos = [[0.05, 0.03, 0.02], [2.25, 2.18, 2.23]][:n_ce]
    spc = [0] * n_ce
    enr = [{"species": 0, "l": l, "a": ex, "rc": 3.0, "re": 0.5} for l in range(4) for ex in (3.0, 0.4)]
    info = [{"name": "Ce", "Z": 12.0, "rloc": 0.3}]
    if extra_h:
        pos.append([2.22, 0.04, 0.03])
        spc.append(1)
        enr.append({"species": 1, "l": 0, "a": 0.8, "rc": 3.0, "re": 0.5})
        info.append({"name": "H", "Z": 1.0, "rloc": 0.4})
    return _problem(cubic(a), (2, 2, 2), 1, pos, spc, info, enr,
                    {"n": 3, "n_ref": 6, "levels": 1, "mode": "geom", "dist": 0.6, "tol": 1e-6},
                    [[0.0, 0.0, 0.0]], 4, "limit_cell_%d%s" % (n_ce, "_h" if extra_h else ""))


def many_groups_cell():
    """A 2^3 trilinear cube (a = 4.4) with one atom halfway between two
    vertices (re = 1.2 reaches both and no other) carrying 24 enrichment
    descriptors: 17 of l = 0, 5 of l = 1 and one each of l = 2 and 3
    (exponents spread over 0.3-3.0), so every element holds 24 groups and 44
    functions on each of two vertices, n_loc = 96 (six 16-row tiles).  Giving
    each l waves of its own would take nine waves of four 16-lane slots, one
    more than a wide work group has: the case where its enrichment schedule
    packs the groups instead."""
    a = 4.4
    enr = []
    for l, m in ((0, 17), (1, 5), (2, 1), (3, 1)):
        for ex in np.geomspace(0.3, 3.0, m) if m > 1 else [1.0]:
            enr.append({"species": 0, "l": l, "a": float(ex), "rc": 3.0, "re": 1.2})
    return _problem(cubic(a), (2, 2, 2), 1, [[1.1, 0.03, 0.02]], [0],
                    [{"name": "X", "Z": 4.0, "rloc": 0.4}], enr,
                    {"n": 3, "n_ref": 6, "levels": 1, "mode": "geom", "dist": 0.6, "tol": 1e-6},
                    [[0.0, 0.0, 0.0]], 4, "many_groups_cell")


def with_bloch_enrichment(prob):
    """A copy of prob whose enrichment functions are Bloch-periodic (eq. Psi
    with f(R) = exp(i k.R)); its PU functions are then periodic and its
    element matrices complex and per k-point."""
    out = copy.deepcopy(prob)
    out["enrichment_phase"] = "bloch"
    out["name"] = prob["name"] + "+bloch"
    return out


def lih_supercell():
    """2x2x2 supercell of the LiH-like cell (a = 15.2, 64 atoms, jittered
    N(0, 0.05) seed 0), 16^3 triquadratic, same rule and enrichments; Gamma."""
    a = 15.2
    red, spc = _lih_reduced(2)
    pos = red * a + jitter(len(spc))
    return _problem(
        cubic(a), [16] * 3, 2, pos, spc, LIH_SPECIES, copy.deepcopy(LIH_ENR),
        {"n": 6, "n_ref": 8, "levels": 2, "mode": "geom", "dist": 1.0, "tol": 1e-6},
        [[0.0, 0.0, 0.0]], 16, "lih_supercell")


def small(kind: str = "lih", mesh=(2, 3, 2), fe_order: int = 2, levels: int = 1,
          n: int = 3, a: float = 5.0, kpts=((0.0, 0.0, 0.0),), re: float = 1.6,
          rc: float = 2.2, lattice=None):
    """Small problems the oracle finishes in well under a second.

    kind = "lih": the LiH-like two-species cell scaled to side a (4 Li + 4 H,
    jittered); kind = "one": a single atom with one s and one p descriptor;
    kind = "ceal": Ce/Al with s..f descriptors (many functions per element).
    """
    if lattice is None:
        lattice = cubic(a)
    lat = np.asarray(lattice, float)
    if kind == "lih":
        red, spc = _lih_reduced(1)
        pos = red @ lat + jitter(len(spc))
        enr = []
        for e in LIH_ENR:
            e = dict(e)
            e["rc"], e["re"] = rc, re
            enr.append(e)
        info = LIH_SPECIES
    elif kind == "one":
        pos = np.array([[0.3, 0.2, 0.1]]) @ lat + 0.0
        spc = [0]
        enr = [{"species": 0, "l": 0, "a": 1.0, "rc": rc, "re": re},
               {"species": 0, "l": 1, "a": 0.7, "rc": rc, "re": re}]
        info = [{"name": "X", "Z": 1.0, "rloc": 0.5}]
    elif kind == "ceal":
        pos = np.array([[0.02, 0.01, 0.03], [0.51, 0.47, 0.55]]) @ lat
        spc = [0, 1]
        enr = []
        for l in range(4):
            for ex in (3.0, 0.4):
                enr.append({"species": 0, "l": l, "a": ex, "rc": rc, "re": re})
        for l in range(3):
            enr.append({"species": 1, "l": l, "a": 0.6, "rc": rc, "re": re})
        info = [{"name": "Ce", "Z": 12.0, "rloc": 0.3}, {"name": "Al", "Z": 3.0, "rloc": 0.3}]
    else:
        raise ValueError(kind)
    return _problem(
        lat, mesh, fe_order, pos, spc, info, enr,
        {"n": n, "n_ref": n + 3, "levels": levels, "mode": "geom", "dist": 1.0,
         "tol": 1e-6},
        list(kpts), 4, f"small-{kind}")



def random_small(seed: int):
    """A seeded random small problem for parity sweeps (the oracle finishes it
    in about a second): kind, mesh, element order, rule depth and Gauss order,
    cell size and shape (a small random shear of a cube; sheared cells take
    the unrefined rule), enrichment radii and two random k-points."""
    rng = np.random.default_rng(1000 + seed)
    kind = ["lih", "one", "ceal"][int(rng.integers(0, 3))]
    mesh = [int(m) for m in rng.integers(2, 4, size=3)]
    if kind == "ceal":
        mesh[2] = 2
    fe_order = int(rng.integers(1, 3))
    n = int(rng.integers(2, 5))
    a = float(rng.uniform(4.4, 5.2))
    skew = bool(rng.integers(0, 2))
    lattice = a * (np.eye(3) + (rng.uniform(-0.06, 0.06, size=(3, 3)) if skew else 0.0))
    levels = 0 if skew else int(rng.integers(0, 2))
    if kind == "ceal":
        rc, re = float(rng.uniform(2.6, 3.0)), float(rng.uniform(2.0, 2.4))
    else:
        rc, re = float(rng.uniform(2.0, 2.4)), float(rng.uniform(1.4, 1.8))
    kpts = [list(map(float, rng.uniform(-0.5, 0.5, size=3))) for _ in range(2)]
    prob = small(kind, mesh=tuple(mesh), fe_order=fe_order, levels=levels, n=n, a=a, kpts=kpts,
                 re=re, rc=rc, lattice=lattice.tolist())
    prob["name"] = f"random-{seed}"
    return prob

def lih_table1(re: float, cells: int = 1, mesh: int = 3, a: float = 4.63):
    """The paper's LiH cubic cell for its sparsity table: Li at 0 (two s-type
    enrichments), H at the body centre (one), a = 4.63 bohr; optionally a
    cells^3 supercell (Li at the corners and H at the body centres of every
    sub-cube)."""
    pos, spc = [], []
    for t3 in range(cells):
        for t2 in range(cells):
            for t1 in range(cells):
                pos.append([t1 * a, t2 * a, t3 * a])
                spc.append(0)
                pos.append([(t1 + 0.5) * a, (t2 + 0.5) * a, (t3 + 0.5) * a])
                spc.append(1)
    enr = [{"species": 0, "l": 0, "a": 1.0, "rc": 2 * a, "re": re},
           {"species": 0, "l": 0, "a": 0.5, "rc": 2 * a, "re": re},
           {"species": 1, "l": 0, "a": 1.0, "rc": 2 * a, "re": re}]
    if re <= 0:
        enr = []
    return _problem(
        cubic(a * cells), [mesh] * 3, 3, pos, spc, LIH_SPECIES, enr,
        {"n": 2, "n_ref": 3, "levels": 0, "mode": "geom", "dist": 0.0, "tol": 1e-6},
        [[0.0, 0.0, 0.0]], 1, f"lih-table1-re{re}")
