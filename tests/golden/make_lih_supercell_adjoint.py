"""Write lih_supercell_adjoint.txt: the adjoint of the assembly (dL/dR of
every atom and dL/dV summed over the points of every element) for the 2x2x2
LiH-like supercell (a = 15.2 bohr, 64 atoms jittered N(0, 0.05 bohr) seed 0,
16^3 triquadratic hexes, 6^3 Gauss points and two octree levels within 1 bohr
of a nucleus), Gamma point, with L = Re sum conj(P_ij) H_ij and the rank-128
adjoint P = C C^H (C from workloads.adjoint_factor, seed 0) on the sparsity
pattern of H; the rule, the enriched sets and V are held fixed (eq. rhoe and
the adjoint of eq. disceig3d).

Only the oracle and the seeded input generators are used: the oracle's
per-element adjoint with P restricted to each element's local functions,
summed over the elements in element order.  Run from the repository root:
python tests/golden/make_lih_supercell_adjoint.py   (the potential at the
12.1 M points takes several minutes on the CPU; the oracle runs on a thread
pool, each call single-threaded).
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lih_supercell_adjoint.txt")


def main():
    prob = W.lih_supercell()
    t0 = time.time()
    o = oracle.Oracle(prob)
    xyz, _, qoff = o.quadrature()
    V = oracle.potential_np(xyz, prob)
    del xyz
    t1 = time.time()
    print(f"rule and potential {t1 - t0:.0f} s", flush=True)
    C = W.adjoint_factor(o.n_dof, rank=128, seed=0)

    def one(e):
        g, _ = o.element_dofs(e)
        Ploc = C[g] @ C[g].conj().T
        dVe, dRe = o.backward_element(e, V[qoff[e]:qoff[e + 1]], (0.0, 0.0, 0.0), Ploc)
        return dVe.sum(), dRe

    threads = max(1, len(os.sched_getaffinity(0)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, range(o.n_elem)))
    dR = np.zeros((o.n_atoms, 3))
    for _, dRe in res:          # element order
        dR += dRe
    t2 = time.time()
    print(f"adjoint {t2 - t1:.0f} s on {threads} threads", flush=True)
    with open(OUT, "w") as f:
        f.write("# Adjoint of the PUFE assembly (eq. rhoe, adjoint of eq. disceig3d) for the 2x2x2\n")
        f.write("# LiH-like supercell: a = 15.2 bohr, 64 atoms jittered N(0, 0.05 bohr) seed 0, 16^3\n")
        f.write("# triquadratic hexes, 6^3 Gauss + 2 octree levels within 1 bohr, Gamma; L = Re<P, H>\n")
        f.write("# with P = C C^H on the pattern of H, C = workloads.adjoint_factor(n_dof, 128, seed 0).\n")
        f.write(f"# FP64 oracle, per-element adjoint summed in element order; n_dof {o.n_dof},\n")
        f.write(f"# n_qp {o.n_qp}.  Written by tests/golden/make_lih_supercell_adjoint.py.\n")
        f.write("# dLdR: atom, x, y, z\n")
        for A in range(o.n_atoms):
            f.write(f"dLdR {A} {dR[A, 0]:.16e} {dR[A, 1]:.16e} {dR[A, 2]:.16e}\n")
        f.write("# dLdV summed over the points of each element: element, sum\n")
        for e, (s, _) in enumerate(res):
            f.write(f"dLdV_sum {e} {s:.16e}\n")
    print("written", OUT)


if __name__ == "__main__":
    main()
