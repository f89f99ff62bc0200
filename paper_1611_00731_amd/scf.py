"""Fixed-point (self-consistent field) iteration of the paper's fig. scf on the
library (section "Self-consistent calculations", eqs. veff, poisson, rhoe).

Each iteration: H and S at every k-point (pufe_assemble), the states of each
k-point occupied with weight 2 / n_k (the dense eigensolve of eq.
disceig3d): the lowest n_el / 2 for an insulator, or Fermi-Dirac occupations
of width sigma around the chemical potential that holds n_el electrons (for
metals and odd electron counts), the electron density at the rule's points from
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


def fermi_occupations(eigenvalues, n_electrons, sigma):
    """Occupations 2 w_k / (1 + exp((eps - mu) / sigma)), w_k = 1 / n_k, with
    the chemical potential mu bisected (200 halvings of [lowest - 40 sigma,
    highest + 40 sigma]) until they sum to n_electrons.  eigenvalues: one
    host array per k-point; returns mu and one occupation array per k-point."""
    allv = np.concatenate(eigenvalues)
    scale = 2.0 / len(eigenvalues)

    def occ(mu):   # 1 / (1 + e^x) = exp(-log(1 + e^x)), safe for large |x|
        return scale * np.exp(-np.logaddexp(0.0, (allv - mu) / sigma))

    lo, hi = float(allv.min()) - 40.0 * sigma, float(allv.max()) + 40.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if float(occ(mid).sum()) < n_electrons else (lo, mid)
    mu = 0.5 * (lo + hi)
    return mu, np.split(occ(mu), np.cumsum([len(e) for e in eigenvalues])[:-1])


def run_scf(p, V_ion, n_electrons, kpts, n_iter, alpha=0.3, n_extra=2, tol=1e-13, smearing=None):
    """p: a set-up Problem; V_ion: the local ionic potential at its points
    (device float64); smearing: the Fermi-Dirac width sigma (Ha), or None for
    doubly occupied lowest states (an even electron count).  Returns V_in
    after n_iter iterations and, per iteration, the lowest ceil(n_el/2) +
    n_extra eigenvalues of every k-point (n_k x m array) and the residual
    (int (V_out - V_in)^2)^(1/2)."""
    import torch

    from . import eigh, pufe_lda_xc

    n_occ = int(np.ceil(n_electrons / 2 - 1e-12))
    if not smearing and abs(2 * n_occ - n_electrons) > 1e-12:
        raise ValueError("an even number of electrons is assumed without smearing (doubly occupied states)")
    _, w, _ = p.quadrature()
    r, c = bsr_index(p.layout())
    rows = torch.from_numpy(r).to(V_ion.device)
    cols = torch.from_numpy(c).to(V_ion.device)
    V = V_ion.clone()
    hist = []
    for _ in range(n_iter):
        dens = torch.zeros_like(V)
        evs = []
        sols = []
        for kap in kpts:
            H, S = p.assemble(V, [tuple(kap)])
            e, Cv = eigh(p.to_dense(H[0]), p.to_dense(S[0]))
            evs.append(e[:n_occ + n_extra])
            sols.append((e, Cv))
        if smearing:
            _, occ = fermi_occupations([e.cpu().numpy() for e, _ in sols], n_electrons, smearing)
        else:
            occ = [np.where(np.arange(len(e)) < n_occ, 2.0 / len(kpts), 0.0) for e, _ in sols]
        for kap, (e, Cv), f in zip(kpts, sols, occ):
            keep = np.nonzero(f > 1e-14 * f.max())[0]
            fk = torch.from_numpy(f[keep]).to(Cv.device)
            Ck = Cv[:, torch.from_numpy(keep).to(Cv.device)]
            Pk = (Ck * fk) @ Ck.mH
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
