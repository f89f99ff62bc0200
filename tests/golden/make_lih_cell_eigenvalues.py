"""Write lih_cell_eigenvalues.txt: the lowest eigenvalues of the discrete
generalized eigenproblem H c = eps S c (eq. disceig3d) for the LiH-like
rock-salt cell (a = 7.6 bohr, 8^3 triquadratic hexes, 6^3 Gauss points and
two octree levels within 1 bohr of a nucleus, Gamma point), assembled by the
FP64 CPU oracle and solved by dense LAPACK (scipy).

Only the oracle and the seeded input generators are used.  Run from the
repository root:  python tests/golden/make_lih_cell_eigenvalues.py
(about two minutes, single thread).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lih_cell_eigenvalues.txt")


def main():
    prob = W.lih_cell()
    m = prob["n_eig"]
    t0 = time.time()
    o = oracle.Oracle(prob)
    xyz, _, _ = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    H, S = o.assemble_dense(V)
    t1 = time.time()
    ev = oracle.generalized_eigh(H.real, S.real, m)
    t2 = time.time()
    with open(OUT, "w") as f:
        f.write("# Lowest eigenvalues (Ha) of H c = eps S c, eq. disceig3d, for the LiH-like\n")
        f.write("# rock-salt cell: a = 7.6 bohr, 4 Li + 4 H jittered N(0, 0.05 bohr) seed 0,\n")
        f.write("# 8^3 triquadratic hexes, 6^3 Gauss + 2 octree levels within 1 bohr, Gamma,\n")
        f.write("# V = -Z erf(r/0.4)/r over images within 12 bohr, enrichments H s(0.8),\n")
        f.write("# Li s(2.0, 0.3) + p(0.5).  FP64 oracle assembly, dense LAPACK solve.\n")
        f.write(f"# written by tests/golden/make_lih_cell_eigenvalues.py; n_dof {o.n_dof}\n")
        for e in ev:
            f.write(f"{e:.15e}\n")
    print(f"assembly {t1 - t0:.1f} s, eigensolve {t2 - t1:.1f} s, n_dof {o.n_dof}")
    print(ev)


if __name__ == "__main__":
    main()
