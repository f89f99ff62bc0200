"""Write ceal_deep_elements.txt: element matrices of the deepest elements of
the CeAl-like CsCl cell (a = 5.8 bohr, 12^3 triquadratic hexes, 8^3 Gauss
points and three octree levels within 1 bohr of a nucleus), eq. disceig3d
restricted to one element:
    H_e[a][b] = sum_q w_q (1/2 grad phi_a . grad phi_b + V_q phi_a phi_b),
    S_e[a][b] = sum_q w_q phi_a phi_b.
The elements: the first fully refined element (512 leaves, 262,144 points)
with the most local functions (283), one with 288 leaves and 283 functions,
and the first fully refined one next to the Al atom (99 functions).  Each
matrix is stored as checks that the tests can compare entry by entry or
vector by vector: the Frobenius norms, the diagonal, the products with a
seeded random vector, and 400 seeded entries.

Only the oracle and the seeded input generators are used.  Run from the
repository root:  python tests/golden/make_ceal_deep_elements.py
(a few minutes; the elements run on a thread pool, each single-threaded).
"""
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from workloads.potential import potential_at  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ceal_deep_elements.txt")
N_ENTRIES = 400


def pick(o):
    _, _, loff = o.leaves()
    nl = np.diff(loff)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    first = lambda m: int(np.nonzero(m)[0][0])
    return [first((nl == 512) & (nloc == nloc.max())), first((nl == 288) & (nloc == nloc.max())),
            first((nl == 512) & (nloc == 99))]


def checks(e, He, Se):
    n = He.shape[0]
    rng = np.random.default_rng(1000 + e)
    x = rng.normal(size=n)
    ab = rng.integers(0, n, size=(N_ENTRIES, 2))
    return {"x": x, "ab": ab, "H": (np.linalg.norm(He), np.diag(He), He @ x, He[ab[:, 0], ab[:, 1]]),
            "S": (np.linalg.norm(Se), np.diag(Se), Se @ x, Se[ab[:, 0], ab[:, 1]])}


def main():
    prob = W.ceal_cell()
    t0 = time.time()
    o = oracle.Oracle(prob)
    elems = pick(o)
    xyz, _, qoff = o.quadrature()
    Vs = {e: potential_at(torch.from_numpy(np.ascontiguousarray(xyz[qoff[e]:qoff[e + 1]])), prob).numpy()
          for e in elems}
    del xyz
    print(f"rule and potential {time.time() - t0:.0f} s; elements {elems}", flush=True)
    with ThreadPoolExecutor(max_workers=len(elems)) as ex:
        mats = list(ex.map(lambda e: o.element_matrices(e, Vs[e]), elems))
    print(f"element matrices {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Element matrices (eq. disceig3d on one element) of the deepest elements of the\n")
        f.write("# CeAl-like CsCl cell: a = 5.8 bohr, 12^3 triquadratic hexes, 8^3 Gauss + 3 octree\n")
        f.write("# levels within 1 bohr, V = -Z erf(r/0.3)/r (Ce 12, Al 3) over images within 12 bohr,\n")
        f.write("# enrichments r_c = 4: Ce s,p,d,f x a = 3.0, 0.4; Al s,p,d a = 0.6; r_e = 2.5.\n")
        f.write("# FP64 oracle.  Written by tests/golden/make_ceal_deep_elements.py.  Per element:\n")
        f.write("# 'element e nloc nq', 'x' (seeded vector, rng seed 1000 + e), 'ab' (seeded entry\n")
        f.write("# indices), then for M in H, S: 'M_fro', 'M_diag', 'M_x' (M @ x), 'M_ab' (entries).\n")
        for e, (He, Se) in zip(elems, mats):
            c = checks(e, He, Se)
            f.write(f"element {e} {He.shape[0]} {qoff[e + 1] - qoff[e]}\n")
            f.write("x " + " ".join(f"{v:.17e}" for v in c["x"]) + "\n")
            f.write("ab " + " ".join(f"{a} {b}" for a, b in c["ab"]) + "\n")
            for M in ("H", "S"):
                fro, dg, mx, ent = c[M]
                f.write(f"{M}_fro {fro:.17e}\n")
                f.write(f"{M}_diag " + " ".join(f"{v:.17e}" for v in dg) + "\n")
                f.write(f"{M}_x " + " ".join(f"{v:.17e}" for v in mx) + "\n")
                f.write(f"{M}_ab " + " ".join(f"{v:.17e}" for v in ent) + "\n")
    print("written", OUT)


if __name__ == "__main__":
    main()
