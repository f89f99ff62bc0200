"""Write lih_cell_projector_coefficients.txt: coefficients of the separable
nonlocal term of eq. disceig3d,
    f_J^i = integral over the cell of conj(phi_i) times the Bloch sum of the
            projector function J,
on the LiH-like cell (a = 7.6 bohr, 8^3 triquadratic hexes, 6^3 Gauss points
and two octree levels within 1 bohr of a nucleus) with its synthetic
projectors (Li: s and p, H: s), for the columns of a sample of basis
functions: every function of the vertex nearest to one Li and to one H atom,
plus seeded random ones.  The nonlocal term on the sample is then
sum_J h_J f_J^i conj(f_J^j).  Two k-points: Gamma and a general one.

Only the oracle and the seeded input generators are used.  Run from the
repository root:  python tests/golden/make_lih_cell_projector_coefficients.py
(about a minute per k-point; the k-points run on two threads).
"""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lih_cell_projector_coefficients.txt")
KPTS = [[0.0, 0.0, 0.0], [0.12, -0.24, 0.37]]
N_RANDOM = 40


def problem():
    return W.with_projectors(W.lih_cell())


def sample_dofs(prob, dof_offset):
    """Functions of the vertex nearest to atom 0 (Li) and to atom 4 (H), then
    N_RANDOM seeded random functions; sorted, unique."""
    n = np.array(prob["mesh"])
    lat = np.array(prob["lattice"], float)
    red = np.array(prob["atoms"], float) @ np.linalg.inv(lat)
    picked = []
    for atom in (0, 4):
        j = np.rint(red[atom] % 1.0 * n).astype(int) % n
        v = (j[2] * n[1] + j[1]) * n[0] + j[0]
        picked.extend(range(dof_offset[v], dof_offset[v + 1]))
    rng = np.random.default_rng(7)
    picked.extend(rng.integers(0, dof_offset[-1], N_RANDOM).tolist())
    return np.unique(np.array(picked, np.int64))


def function_weights(prob):
    """h_J in the order of the coefficients: projector descriptor, then atom
    of its species, then m = -l..l."""
    h = []
    for q in prob["projectors"]:
        for s in prob["species"]:
            if s == q["species"]:
                h.extend([q["h"]] * (2 * q["l"] + 1))
    return np.array(h)


def main():
    prob = problem()
    o = oracle.Oracle(prob)
    idx = sample_dofs(prob, o.dof_offset())
    h = function_weights(prob)
    t0 = time.time()

    def one(kap):
        return oracle.Oracle(prob).nonlocal_f(kap)

    with ThreadPoolExecutor(len(KPTS)) as ex:
        Fs = list(ex.map(one, KPTS))
    assert all(F.shape == (len(h), o.n_dof) for F in Fs)
    with open(OUT, "w") as f:
        f.write("# Projector coefficients f_J^i of the separable nonlocal term (eq. disceig3d)\n")
        f.write("# LiH-like cell + synthetic projectors; FP64 CPU oracle, "
                "tests/golden/make_lih_cell_projector_coefficients.py\n")
        f.write(f"# n_dof {o.n_dof} n_fun {len(h)} n_sample {len(idx)} n_k {len(KPTS)}\n")
        f.write("sample " + " ".join(map(str, idx)) + "\n")
        f.write("h " + " ".join(f"{x:.17e}" for x in h) + "\n")
        for kap, F in zip(KPTS, Fs):
            f.write("k " + " ".join(f"{x:.17e}" for x in kap) + "\n")
            for J in range(len(h)):
                row = F[J, idx]
                f.write(" ".join(f"{z.real:.17e} {z.imag:.17e}" for z in row) + "\n")
    print(f"wrote {OUT}: {len(idx)} functions, {len(h)} projector functions, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
