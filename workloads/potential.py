"""Synthetic local potential for the workloads (an input of the path).

V(x) = sum_A sum_images -Z_A erf(r / rloc_A) / r, with r = |x - tau_A - n.a|
and an image counted iff r <= cutoff (12 bohr in every workload).  This is a
stand-in for a self-consistent Kohn-Sham potential; the assembly treats V as
given values at the quadrature points.  Evaluated with torch in float64 on
whatever device the points live on.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _image_range(lat, inv, tau, cutoff):
    # every image within `cutoff` of a point of the unit cell
    rad = cutoff * np.linalg.norm(inv, axis=0)
    u = tau @ inv
    lo = np.floor(-u - rad).astype(int) - 1
    hi = np.ceil(1.0 - u + rad).astype(int) + 1
    return lo, hi


def potential_at(points: torch.Tensor, prob: dict, chunk: int = 1 << 20) -> torch.Tensor:
    """V at Cartesian points (n x 3 float64 tensor), same device."""
    lat = np.asarray(prob["lattice"], float)
    inv = np.linalg.inv(lat)
    cutoff = float(prob.get("potential", {}).get("cutoff", 12.0))
    out = torch.zeros(points.shape[0], dtype=torch.float64, device=points.device)
    two_over_sqrtpi = 2.0 / math.sqrt(math.pi)
    for A, tau in enumerate(np.asarray(prob["atoms"], float)):
        sp = prob["species_info"][prob["species"][A]]
        Z, rl = float(sp["Z"]), float(sp["rloc"])
        lo, hi = _image_range(lat, inv, tau, cutoff)
        centres = []
        for n3 in range(lo[2], hi[2] + 1):
            for n2 in range(lo[1], hi[1] + 1):
                for n1 in range(lo[0], hi[0] + 1):
                    centres.append(tau + n1 * lat[0] + n2 * lat[1] + n3 * lat[2])
        centres = torch.tensor(np.array(centres), dtype=torch.float64, device=points.device)
        for s in range(0, points.shape[0], chunk):
            p = points[s:s + chunk]
            for c in centres:
                r = torch.linalg.vector_norm(p - c, dim=1)
                t = r / rl
                small = t < 1e-3
                safe_r = torch.where(small, torch.ones_like(r), r)
                v = -Z * torch.erf(t) / safe_r
                vs = -Z * two_over_sqrtpi / rl * (1.0 - t * t / 3.0 + t ** 4 / 10.0)
                v = torch.where(small, vs, v)
                out[s:s + chunk] += torch.where(r <= cutoff, v, torch.zeros_like(v))
    return out
