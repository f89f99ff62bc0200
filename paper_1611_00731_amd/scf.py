"""Fixed-point (self-consistent field) iteration of the paper's fig. scf on the
library (section "Self-consistent calculations", eqs. veff, poisson, rhoe).

Each iteration: H and S at every k-point (pufe_assemble), the lowest
n_el / 2 states of each doubly occupied with weight 2 / n_k (the dense
eigensolve of eq. disceig3d), the electron density at the rule's points from
the adjoint with P = sum_i f_i c_i c_i^H (pufe_assemble_backward gives
w_q n(x_q)), V_out = V_ion + V_H[n] + V_xc[n] (pufe_hartree, pufe_lda_xc),
and the linear mix V_in += alpha (V_out - V_in).  The local ionic potential
V_ion at the points is an input; the enrichment is the periodic form.
"""
from __future__ import annotations

import numpy as np


def bsr_index(layout):
    """Global (row, col) DOF of every stored BSR entry, in value order."""
    off, rp, bc = layout["dof_offset"], layout["brow_ptr"], layout["bcol"]
    rows, cols = [], []
    for v in range(len(rp) - 1):
        bv = off[v + 1] - off[v]
        for k in range(rp[v], rp[v + 1]):
            w = bc[k]
            bw = off[w + 1] - off[w]
            rows.append(np.repeat(np.arange(off[v], off[v + 1]), bw))
            cols.append(np.tile(np.arange(off[w], off[w + 1]), bv))
    return np.concatenate(rows), np.concatenate(cols)


def run_scf(p, V_ion, n_electrons, kpts, n_iter, alpha=0.3, n_extra=2, tol=1e-13):
    """p: a set-up Problem; V_ion: the local ionic potential at its points
    (device float64).  Returns V_in after n_iter iterations and, per
    iteration, the lowest n_el/2 + n_extra eigenvalues of every k-point
    (n_k x m array) and the residual (int (V_out - V_in)^2)^(1/2)."""
    import torch

    from . import eigh, pufe_lda_xc

    n_occ = int(round(n_electrons / 2))
    if abs(2 * n_occ - n_electrons) > 1e-12:
        raise ValueError("an even number of electrons is assumed (doubly occupied states)")
    _, w, _ = p.quadrature()
    r, c = bsr_index(p.layout())
    rows = torch.from_numpy(r).to(V_ion.device)
    cols = torch.from_numpy(c).to(V_ion.device)
    V = V_ion.clone()
    hist = []
    for _ in range(n_iter):
        dens = torch.zeros_like(V)
        evs = []
        for kap in kpts:
            H, S = p.assemble(V, [tuple(kap)])
            e, Cv = eigh(p.to_dense(H[0]), p.to_dense(S[0]))
            evs.append(e[:n_occ + n_extra])
            Co = Cv[:, :n_occ]
            Pk = (2.0 / len(kpts)) * (Co @ Co.mH)
            dV, _ = p.backward(V, tuple(kap), Pk[rows, cols].contiguous(), want_dR=False)
            dens += dV / w
        vh, _, _, _ = p.hartree(dens, tol)
        vxc = torch.empty_like(dens)
        pufe_lda_xc(dens, vxc)
        Vout = V_ion + vh + vxc
        res = float(torch.sqrt(torch.dot(w, (Vout - V) ** 2)))
        hist.append((torch.stack(evs).cpu().numpy(), res))
        V = V + alpha * (Vout - V)
    return V, hist
