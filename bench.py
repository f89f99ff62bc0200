"""Benchmark of the PUFE H/S assembly on one MI355X.

Headline workload: the CeAl-like CsCl cell (a = 5.8 bohr, Ce at the origin,
Al at the body centre, 12^3 triquadratic hexes, 8^3 Gauss points + 3
geometric octree levels within 1 bohr of a nucleus, 1728 elements, 27.3 M
quadrature points, 41 enrichment functions per Ce-Al pair, n_loc up to 283,
N = 37,891) at the 4 time-reversal-reduced 2x2x2 Monkhorst-Pack k-points,
complex128 H and S, FP64, autotuned.  It is the largest configuration that
fits one GPU.  One step = one full assembly of H and S from V at the
quadrature points: the fused basis-evaluation + MFMA element contraction, the
K-chunk sum and the coloured Bloch scatter into block-sparse H and S for the
4 k-points.  Inputs are resident in HBM before timing starts; the rule (built
once per geometry) is set up outside the timed region.

Prints one JSON line (rank 0): elements/s (elements x k-points per second),
ms/step, the contraction kernel's MFMA roofline fraction (algorithmic flops
per launch over its average launch time measured with HIP events on the
launch stream), the split-BF16 forms on the same inputs, and the CPU oracle
timed on a bounded, stratified element sample of the same workload.  Further
legs (extra): the LiH-like cell with the eigenvalue error of the assembled
matrices against the stored FP64 oracle eigenvalues, the lattice-constant
sweep batch and the adjoint on the 64-atom supercell.

Environment: PUFE_TUNE_CACHE, an optional file where the autotuner keeps its
choice per problem shape and device (absent: the tuner runs every time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "enriched H/S assembly elements/s + MFMA util; eig err vs FP64 oracle (Ha)"
PEAK = {"fp64": 78.6, "bf16x3": 2500.0 / 3, "bf16x6": 2500.0 / 6}   # TFLOP/s, dense
HBM_PEAK_GBS = 8000.0


# Figures of rocprofv3 counter passes over the contraction kernel (HBM bytes
# from FETCH_SIZE / WRITE_SIZE scaled by a plain device copy; MFMA busy cycles
# and executed MFMA flops), per workload.  Each is reported only while the
# kernel sources it was measured on are unchanged (their SHA-256 is recorded
# next to the figure).
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["kernels.hip", "stage.hpp", "tables.hpp", "enrich.hpp", "basis.hpp", "device_common.hpp",
                  "capi.cpp", "plan.cpp"]


def kernel_sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_00731_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded(fname, *keys):
    """Values of `keys` recorded in profiles/<fname> for the current kernel
    sources (None for each when absent or measured on other sources)."""
    path = os.path.join(PROFILES, fname)
    if not os.path.exists(path):
        return [None] * len(keys)
    txt = open(path).read()
    m_h = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", txt)
    if not m_h or m_h.group(1) != kernel_sources_digest():
        return [None] * len(keys)
    out = []
    for k in keys:
        m = re.search(k + r":\s*([0-9.eE+-]+)", txt)
        out.append(float(m.group(1)) if m else None)
    return out


# Lowest eigenvalues of the LiH-like cell from the FP64 CPU oracle (dense
# assembly, LAPACK solve), written by tests/golden/make_lih_cell_eigenvalues.py.
GOLDEN_EIGS = os.path.join(ROOT, "tests", "golden", "lih_cell_eigenvalues.txt")


def golden_eigenvalues():
    import numpy as np
    return np.loadtxt(GOLDEN_EIGS, comments="#")


def eig_error(P, p, H, S, ev_ref):
    """max |eps - eps_oracle| (Ha) over the lowest eigenvalues of the
    assembled Gamma-point H, S (device FP64 Cholesky + Hermitian solve);
    None with the reason when S is not numerically positive definite."""
    import numpy as np
    Hd = p.to_dense(H[0]).real.contiguous()
    Sd = p.to_dense(S[0]).real.contiguous()
    try:
        ev = P.eig(Hd, Sd, len(ev_ref)).cpu().numpy()
    except RuntimeError as e:
        return None, str(e).splitlines()[0][:120]
    return float(np.abs(ev - ev_ref).max()), None


def copy_probe(mib=1024, reps=3):
    """A plain device copy of known size, the scale for the PMC byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64).to("cuda")   # host fill, then a plain upload
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "reps": reps}),
          flush=True)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def element_work(prob, sizes, layout, leaf_off, n3):
    """(n_loc, n_q) per element and the algorithmic flops 5 n_q n_loc (n_loc+1)
    of the symmetric H + S contractions."""
    import numpy as np
    n1, n2, n3m = prob["mesh"]
    nfs = sizes["n_fe_slots"]
    nfe = 8 if prob["fe_order"] == 1 else 27
    nenr = np.diff(layout["dof_offset"]) - nfs
    e = np.arange(sizes["n_elem"])
    i1, i2, i3 = e % n1, (e // n1) % n2, e // (n1 * n2)
    nloc = np.full(e.shape, nfe)
    for c in range(8):
        j1 = (i1 + (c & 1)) % n1
        j2 = (i2 + ((c >> 1) & 1)) % n2
        j3 = (i3 + ((c >> 2) & 1)) % n3m
        nloc = nloc + nenr[(j3 * n2 + j2) * n1 + j1]
    nq = np.diff(leaf_off) * n3
    flops = 5.0 * nq * nloc * (nloc + 1)
    return nloc, nq, flops


def time_assembly(P, p, V, kpts, precision, H, S, steps, warmup):
    """(ms per step without per-kernel events, [contraction, scatter, chunk
    sum] ms per launch from a second, instrumented run of the same steps)."""
    import torch
    st = torch.cuda.current_stream()
    for _ in range(warmup):
        P.pufe_assemble(p.ctx, V, kpts, precision, "c128", H, S)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(st)
    for _ in range(steps):
        P.pufe_assemble(p.ctx, V, kpts, precision, "c128", H, S)
    t1.record(st)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # per-kernel durations from HIP events recorded by the library around each
    # of its kernels on the launch stream (the event records between the
    # kernels would lower the step throughput, hence a second run)
    P.pufe_enable_timing(p.ctx, True)
    P.pufe_kernel_times(p.ctx, reset=True)
    t0.record(st)
    for _ in range(steps):
        P.pufe_assemble(p.ctx, V, kpts, precision, "c128", H, S)
    t1.record(st)
    torch.cuda.synchronize()
    ms_instr = t0.elapsed_time(t1) / steps
    kms, kc = P.pufe_kernel_times(p.ctx, reset=True)
    P.pufe_enable_timing(p.ctx, False)
    per = [kms[i] / max(kc[i], 1) for i in range(4)]
    return ms, ms_instr, {"contract_ms": per[0], "scatter_ms_per_assembly": kms[1] / steps,
                          "chunk_reduce_ms": per[3]}


def cpu_baseline(prob, n_k, max_threads=16):
    """The oracle's element matrices timed on a stratified sample of the
    workload's elements, extrapolated to the whole cell by the oracle's cost
    per point and local-function pair of each n_loc class; single thread and
    a thread pool over elements (the unchanged single-threaded oracle called
    through ctypes, which releases the GIL)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import oracle
    from workloads.potential import potential_at
    o = oracle.Oracle(prob)
    xyz, _, qp_off = o.quadrature()
    _, _, loff = o.leaves()
    nleaf = np.diff(loff)
    nq = np.diff(qp_off)
    nloc = np.array([o.element_dofs(e)[0].size for e in range(o.n_elem)])
    work = nq.astype(float) * nloc.astype(float) ** 2
    # strata: one unrefined element of every n_loc class, and the cheapest
    # refined element of a class when it runs in a few seconds
    sample = []
    for c in np.unique(nloc):
        m = np.nonzero((nleaf == 1) & (nloc == c))[0]
        if m.size:
            sample.append(int(m[0]))
    rate_guess = 8e-9
    for c in np.unique(nloc[nleaf > 1]):
        m = np.nonzero((nleaf > 1) & (nloc == c))[0]
        e = int(m[np.argmin(work[m])])
        if work[e] * rate_guess < 6.0:
            sample.append(e)
    Vs = {e: potential_at(torch.from_numpy(np.ascontiguousarray(xyz[qp_off[e]:qp_off[e + 1]])), prob).numpy()
          for e in sample}
    del xyz
    t_el = {}
    for e in sample:
        t0 = time.perf_counter()
        o.element_matrices(e, Vs[e])
        t_el[e] = time.perf_counter() - t0
    # cost per point and pair for each (n_loc, refined) class, falling back to
    # the unrefined rate of the same n_loc
    rate = {}
    for e in sample:
        rate[(int(nloc[e]), bool(nleaf[e] > 1))] = t_el[e] / work[e]
    T1 = 0.0
    for e in range(o.n_elem):
        key = (int(nloc[e]), bool(nleaf[e] > 1))
        r = rate.get(key, rate.get((key[0], False)))
        T1 += r * work[e]
    t_sample = sum(t_el.values())
    # the same sample on a pool of threads, every thread running the whole sample
    threads = max(1, min(len(os.sched_getaffinity(0)), max_threads))
    tasks = [e for _ in range(threads) for e in sample]
    tasks.sort(key=lambda e: -work[e])
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda e: o.element_matrices(e, Vs[e]), tasks))
    wall = time.perf_counter() - t0
    speedup = threads * t_sample / wall
    Tn = T1 / speedup
    n_el = o.n_elem
    desc = (f"element matrices (H_e, S_e) of {len(sample)} elements: one unrefined element of each of the "
            f"{len(np.unique(nloc))} n_loc classes and the cheapest refined element of each refined class that "
            f"runs in seconds ({sum(1 for e in sample if nleaf[e] > 1)} refined); every element of the cell "
            f"extrapolated by its class's measured seconds per (point x n_loc^2) "
            f"(EXTRAPOLATED: {T1:.0f} s single-thread for the whole cell; the sample took {t_sample:.1f} s); "
            f"the oracle's element matrices serve all {n_k} k-points (its phase scatter is not counted)")
    return {"value": n_el * n_k / Tn, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": desc + f"; {threads} threads over the sample, {wall:.1f} s wall, speed-up {speedup:.2f}",
            "single_thread": {"value": n_el * n_k / T1, "cores": 1, "extrapolated_s": T1,
                              "sample_s": t_sample}}


def bsr_rows_cols(lay):
    """Global (row, col) DOF of every stored BSR value, in value order."""
    import numpy as np
    off, rp, bc = lay["dof_offset"], lay["brow_ptr"], lay["bcol"]
    rows, cols = [], []
    for v in range(len(rp) - 1):
        bv = off[v + 1] - off[v]
        for k in range(rp[v], rp[v + 1]):
            w = bc[k]
            bw = off[w + 1] - off[w]
            rows.append(np.repeat(np.arange(off[v], off[v + 1]), bw))
            cols.append(np.tile(np.arange(off[w], off[w + 1]), bv))
    return np.concatenate(rows), np.concatenate(cols)


def leg_batch(tune_cache, reps=5):
    """The persistent, graph-captured batch over the lattice-constant sweep
    (11 LiH-like cells a = 6.8 .. 8.4 bohr x 8 Monkhorst-Pack k-points, 88
    H and S): each cell tuned first, then replays timed with HIP events, FP64
    with complex128 outputs and bf16x6 with complex64 outputs (errors of the
    latter against the former)."""
    import torch
    import paper_1611_00731_amd as P
    import workloads as W
    from workloads.potential import potential_at
    probs, kpts = W.lih_lattice_sweep(), W.mp2()
    ps, Vs, flops, nel = [], [], 0.0, 0
    for pr in probs:
        p = P.Problem(pr).setup()
        P.pufe_tune(p.ctx, "fp64", tune_cache)
        xyz, _, _ = p.quadrature()
        Vs.append(potential_at(xyz, pr))
        lay = p.layout()
        _, _, leaf_off = p.leaves()
        _, _, f = element_work(pr, p.sizes, lay, leaf_off, pr["quad"]["n"] ** 3)
        flops += float(f.sum())
        nel += p.sizes["n_elem"]
        ps.append(p)
    b = P.Batch(ps)
    st = torch.cuda.current_stream()
    out = {"workload": "11 lattice constants x 8 k-points (88 outputs), one graph replay, each cell tuned"}
    ref = None
    for prec, dt in (("fp64", "c128"), ("bf16x6", "c64")):
        Hs, Ss = b.alloc(len(kpts), out_dtype=dt, device="cuda")
        b.assemble(Vs, kpts, Hs, Ss, precision=prec, out_dtype=dt)            # capture
        b.assemble(Vs, kpts, Hs, Ss, precision=prec, out_dtype=dt)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(st)
        for _ in range(reps):
            b.assemble(Vs, kpts, Hs, Ss, precision=prec, out_dtype=dt)
        t1.record(st)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        row = {"ms": ms, "elements_per_s": nel * len(kpts) / (ms * 1e-3),
               "unique_contractions_per_s": nel / (ms * 1e-3),
               "alg_tflops_whole_batch": flops / (ms * 1e-3) / 1e12,
               "frac_of_peak_whole_batch": flops / (ms * 1e-3) / 1e12 / PEAK[prec]}
        if ref is None:
            ref = (Hs, Ss)
        else:
            row["H_rel_err_vs_fp64"] = max(rel_err(h.double(), r) for h, r in zip(Hs, ref[0]))
            row["S_rel_err_vs_fp64"] = max(rel_err(s_.double(), r) for s_, r in zip(Ss, ref[1]))
        out[prec + "_" + dt] = row
    b.close()
    for p in ps:
        p.close()
    return out


def leg_backward(reps=3):
    """assemble_backward on the 2x2x2 LiH-like supercell (64 atoms, 4096
    elements, 12.1 M points) with a rank-128 Hermitian PSD adjoint P on the
    pattern: dL/dV at every point and dL/dR for all atoms, FP64 and both split
    forms (errors against the FP64 result)."""
    import numpy as np
    import torch
    import paper_1611_00731_amd as P
    import workloads as W
    from workloads.potential import potential_at
    prob = W.lih_supercell()
    p = P.Problem(prob).setup()
    xyz, _, _ = p.quadrature()
    V = potential_at(xyz, prob)
    lay = p.layout()
    _, _, leaf_off = p.leaves()
    nloc, nq, _ = element_work(prob, p.sizes, lay, leaf_off, prob["quad"]["n"] ** 3)
    Cd = torch.from_numpy(W.adjoint_factor(p.sizes["n_dof"], rank=128, seed=0)).cuda()
    rows, cols = bsr_rows_cols(lay)
    rows_d, cols_d = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    Pb = torch.empty(len(rows), dtype=torch.complex128, device="cuda")
    for s0 in range(0, len(rows), 1 << 20):
        r, c = rows_d[s0:s0 + (1 << 20)], cols_d[s0:s0 + (1 << 20)]
        Pb[s0:s0 + (1 << 20)] = (Cd[r] * Cd[c].conj()).sum(-1)
    del Cd, rows_d, cols_d
    st = torch.cuda.current_stream()
    # P~ [grad phi; phi] at every point: 8 n_q n_loc^2 flops
    flops = float((8.0 * nq * nloc.astype(float) ** 2).sum())

    def timed(prec):
        dV, dR = p.backward(V, (0.0, 0.0, 0.0), Pb, None, precision=prec)
        torch.cuda.synchronize()
        P.pufe_enable_timing(p.ctx, True)
        P.pufe_kernel_times(p.ctx, reset=True)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(st)
        for _ in range(reps):
            p.backward(V, (0.0, 0.0, 0.0), Pb, None, precision=prec)
        t1.record(st)
        torch.cuda.synchronize()
        kms, kc = P.pufe_kernel_times(p.ctx, reset=True)
        P.pufe_enable_timing(p.ctx, False)
        return dV, dR, t0.elapsed_time(t1) / reps, kms[2] / max(kc[2], 1)

    dV, dR, ms, kern = timed("fp64")
    out = {"workload": "64-atom LiH-like supercell, 4096 elements, rank-128 adjoint, dL/dV + dL/dR",
           "ms": ms, "adjoint_kernels_ms": kern, "elements_per_s": p.sizes["n_elem"] / (ms * 1e-3),
           "alg_flops": flops, "alg_tflops_adjoint_kernels": flops / (kern * 1e-3) / 1e12,
           "frac_of_fp64_peak": flops / (kern * 1e-3) / 1e12 / PEAK["fp64"]}
    # split-precision forms of U = P~ B, errors against the FP64 result
    for prec in ("bf16x6", "bf16x3"):
        dVs, dRs, ms_s, kern_s = timed(prec)
        out[prec] = {"ms": ms_s, "adjoint_kernels_ms": kern_s,
                     "alg_tflops_adjoint_kernels": flops / (kern_s * 1e-3) / 1e12,
                     "dLdV_rel_err_vs_fp64": float((dVs - dV).norm() / dV.norm()),
                     "dLdR_max_err_rel_vs_fp64": float((dRs - dR).abs().max() / dR.abs().max())}
    p.close()
    return out


def leg_nonlocal(P, W, potential_at, steps=10, warmup=2):
    """The LiH-like cell with its synthetic separable projectors (Li: s and p,
    H: s; eq. disceig3d): whole FP64 assembly with the nonlocal term against
    the same assembly without it, and the projector-coefficient kernels."""
    import torch
    base = W.lih_cell()
    out = {"workload": "LiH-like cell (512 elements, 1.52 M points) with Li s+p and H s projectors, Gamma, "
                       "H+S complex128, FP64"}
    for tag, prob in (("local", base), ("nonlocal", W.with_projectors(base))):
        p = P.Problem(prob).setup()
        xyz, _, _ = p.quadrature()
        V = potential_at(xyz, prob)
        del xyz
        sz = p.sizes
        kpts = prob["kpts"]
        H = torch.empty((len(kpts), sz["nnz"], 2), dtype=torch.float64, device="cuda")
        S = torch.empty_like(H)
        ms, _, _ = time_assembly(P, p, V, kpts, "fp64", H, S, steps, warmup)
        row = {"ms_per_step": ms, "nnz": sz["nnz"]}
        if tag == "nonlocal":
            P.pufe_enable_timing(p.ctx, True)
            P.pufe_kernel_times(p.ctx, reset=True)
            for _ in range(steps):
                P.pufe_assemble(p.ctx, V, kpts, "fp64", "c128", H, S)
            torch.cuda.synchronize()
            kms, kc = P.pufe_kernel_times(p.ctx, reset=True)
            P.pufe_enable_timing(p.ctx, False)
            row["projector_coefficient_kernels_ms"] = kms[4] / steps
            row["scatter_and_nonlocal_update_ms"] = kms[1] / steps
            row["n_projector_functions"] = sum((2 * q["l"] + 1) * prob["species"].count(q["species"])
                                               for q in prob["projectors"])
        out[tag] = row
        del H, S
        p.close()
    out["nonlocal_extra_ms"] = out["nonlocal"]["ms_per_step"] - out["local"]["ms_per_step"]
    out["extra_nnz"] = out["nonlocal"]["nnz"] - out["local"]["nnz"]
    return out


def leg_bloch(P, W, potential_at, steps=5, warmup=1):
    """The LiH-like cell with Bloch-periodic enrichment (eq. Psi with
    f(R) = exp(i k.R)) at 4 k-points, FP64 and bf16x6: every element is
    contracted once per k-point with a real and an imaginary row per enriched
    function, against the periodic form (one contraction for all k-points)."""
    import numpy as np
    import torch
    base = W.lih_cell()
    kpts = [[0.25, 0.25, 0.25], [0.25, 0.25, -0.25], [0.25, -0.25, 0.25], [0.25, -0.25, -0.25]]
    out = {"workload": "LiH-like cell (512 elements, 1.52 M points), 4 k-points, H+S complex128"}
    for tag, prob in (("periodic", base), ("bloch", W.with_bloch_enrichment(base))):
        p = P.Problem(prob).setup()
        xyz, _, _ = p.quadrature()
        V = potential_at(xyz, prob)
        del xyz
        sz = p.sizes
        H = torch.empty((len(kpts), sz["nnz"], 2), dtype=torch.float64, device="cuda")
        S = torch.empty_like(H)
        row = {}
        for prec in ("fp64", "bf16x6"):
            ms, _, kern = time_assembly(P, p, V, kpts, prec, H, S, steps, warmup)
            row[prec] = {"ms_per_step": ms, "contract_ms_per_launch": kern["contract_ms"]}
        if tag == "bloch":
            _, _, loff = P.pufe_get_leaves(p.ctx)
            nloc, nq, _ = element_work(base, sz, p.layout(), loff, p.prob["quad"]["n"] ** 3)
            nfe = 8 if base["fe_order"] == 1 else 27
            rows = 2 * nloc - nfe          # FE rows, and a real and an imaginary row per enriched function
            flops = float(np.sum(5.0 * nq * rows * (rows + 1)))
            c = row["fp64"]["contract_ms_per_launch"]
            row["alg_flops_per_k"] = flops
            row["fp64_contract_tflops"] = flops / (c * 1e-3) / 1e12
            row["fp64_contract_frac_of_peak"] = row["fp64_contract_tflops"] / 78.6
            row["max_rows"] = int(rows.max())
        out[tag] = row
        del H, S
        p.close()
    out["bloch_over_periodic_fp64"] = out["bloch"]["fp64"]["ms_per_step"] / out["periodic"]["fp64"]["ms_per_step"]
    return out


def leg_scf(P, W, potential_at, n_iter=3):
    """Fixed-point iterations (fig. scf) on the LiH-like cell at Gamma: the
    time per iteration and its pieces (assembly, dense eigensolve, density
    from the adjoint, Hartree solve, LDA) from a separately timed pass."""
    import time

    import torch
    from paper_1611_00731_amd.scf import bsr_index, run_scf
    prob = W.lih_cell()
    p = P.Problem(prob).setup()
    xyz, w, _ = p.quadrature()
    V = potential_at(xyz, prob)
    del xyz
    n_el = sum(prob["species_info"][s]["Z"] for s in prob["species"])
    kpts = prob["kpts"]
    run_scf(p, V, n_el, kpts, 1)   # warm-up (builds the Poisson operator)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, hist = run_scf(p, V, n_el, kpts, n_iter)
    torch.cuda.synchronize()
    ms_iter = (time.perf_counter() - t0) * 1e3 / n_iter

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t) * 1e3

    (H, S), t_asm = timed(lambda: p.assemble(V, [tuple(kpts[0])]))
    (e, Cv), t_eig = timed(lambda: P.eigh(p.to_dense(H[0]), p.to_dense(S[0])))
    r, c = bsr_index(p.layout())
    rows, cols = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
    n_occ = int(round(n_el / 2))
    Pk = 2.0 * (Cv[:, :n_occ] @ Cv[:, :n_occ].mH)
    Pb = Pk[rows, cols].contiguous()
    (dV, _), t_den = timed(lambda: p.backward(V, tuple(kpts[0]), Pb, want_dR=False))
    dens = dV / w
    (vh, _, it, res), t_h = timed(lambda: p.hartree(dens))
    vxc = torch.empty_like(dens)
    _, t_xc = timed(lambda: P.pufe_lda_xc(dens, vxc))
    out = {"workload": "LiH-like cell (512 elements, 1.52 M points, %d DOFs), Gamma, %d electrons"
                       % (p.sizes["n_dof"], int(n_el)),
           "ms_per_iteration": ms_iter, "residuals": [h[1] for h in hist],
           "pieces_ms": {"assemble": t_asm, "dense_eigensolve": t_eig, "density_adjoint": t_den,
                         "hartree": t_h, "lda": t_xc},
           "hartree_cg_iterations": it, "hartree_rel_residual": res,
           "electrons_from_density": float(torch.dot(w, dens))}
    p.close()
    return out


def rel_err(A, B):
    return float((A - B).norm() / B.norm())


def leg_ceal_split(P, p, V, kpts, flops, H64, S64):
    """The split-BF16 contractions on the headline inputs: kernel time, rate
    against the effective peak and the relative Frobenius error of H and S
    against the FP64 GPU result."""
    import torch
    out = {}
    H = torch.empty_like(H64)
    S = torch.empty_like(S64)
    for prec in ("bf16x6", "bf16x3"):
        ms, _, k = time_assembly(P, p, V, kpts, prec, H, S, steps=3, warmup=1)
        cms = k["contract_ms"]
        out[prec] = {"ms_per_step": ms, "contract_ms": cms,
                     "alg_tflops": flops / (cms * 1e-3) / 1e12,
                     "frac_of_effective_peak": flops / (cms * 1e-3) / 1e12 / PEAK[prec],
                     "speedup_vs_fp64_contraction": None,
                     "H_rel_err_vs_fp64": rel_err(H, H64), "S_rel_err_vs_fp64": rel_err(S, S64)}
    return out


def leg_lih_cell(P, W, potential_at, steps, warmup, tune_cache, do_eig):
    """The LiH-like cell (a = 7.6 bohr, 8^3 triquadratic hexes, 6^3 Gauss + 2
    octree levels, 512 elements, 1.52 M points, N = 4888), Gamma, complex128:
    assembly rate, contraction roofline and the eigenvalue error of the
    assembled matrices against the stored FP64 oracle eigenvalues, FP64 and
    both split forms."""
    import torch
    prob = W.lih_cell()
    p = P.Problem(prob).setup()
    P.pufe_tune(p.ctx, "fp64", tune_cache)
    sz = p.sizes
    xyz, _, _ = p.quadrature()
    V = potential_at(xyz, prob)
    del xyz
    lay = p.layout()
    _, _, leaf_off = p.leaves()
    _, _, flops = element_work(prob, sz, lay, leaf_off, prob["quad"]["n"] ** 3)
    alg = float(flops.sum())
    kpts = prob["kpts"]
    H = torch.empty((len(kpts), sz["nnz"], 2), dtype=torch.float64, device="cuda")
    S = torch.empty_like(H)
    ev_ref = golden_eigenvalues()
    out = {"workload": "LiH-like rock-salt cell a=7.6 bohr, 8^3 triquadratic hexes, 6^3 Gauss + 2 octree levels "
                       "within 1 bohr, Gamma, H+S complex128",
           "n_elem": sz["n_elem"], "n_qp": sz["n_qp"], "n_dof": sz["n_dof"], "nnz": sz["nnz"],
           "alg_flops": alg}
    eig = {"n_eig": int(len(ev_ref)), "unit": "Ha",
           "reference": "FP64 CPU oracle, dense LAPACK solve (tests/golden/lih_cell_eigenvalues.txt)",
           "note": "bf16x3 keeps two bf16 limbs (about 16 significant bits per operand): its H and S "
                   "errors are near 2e-6, over the 1e-7 split target, and S loses positive "
                   "definiteness at this size; only bf16x6 meets the split targets"}
    for prec in ("fp64", "bf16x6", "bf16x3"):
        ms, ms_i, k = time_assembly(P, p, V, kpts, prec, H, S, steps if prec == "fp64" else 5, warmup)
        cms = k["contract_ms"]
        row = {"ms_per_step": ms, "elements_per_s": sz["n_elem"] * len(kpts) / (ms * 1e-3), "contract_ms": cms,
               "alg_tflops": alg / (cms * 1e-3) / 1e12, "frac_of_peak": alg / (cms * 1e-3) / 1e12 / PEAK[prec]}
        if prec == "fp64":
            row.update(k)
            row["ms_per_step_with_kernel_events"] = ms_i
        out[prec] = row
        if do_eig:
            err, why = eig_error(P, p, H, S, ev_ref)
            eig[prec] = err
            if why:
                eig[prec + "_note"] = why
            log(f"LiH-like eigenvalue error {prec}: {err}")
    if do_eig:
        out["eig_err"] = eig
    p.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=sorted(PEAK))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the LiH-like, batch (lattice sweep) and adjoint measurement legs")
    ap.add_argument("--no-split", action="store_true", help="skip the split-BF16 forms of the headline")
    ap.add_argument("--host-inputs", action="store_true",
                    help="evaluate the synthetic V on the host and copy it over (no torch kernels; "
                         "for hardware-counter runs); implies --no-eig")
    ap.add_argument("--no-eig", action="store_true",
                    help="skip the device eigensolves of the eigenvalue-error fields (the dense "
                         "solver library does not run under hardware-counter collection)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (scale for the PMC byte counters)")
    ap.add_argument("--workload", default="ceal", choices=["ceal", "lih"],
                    help="configuration of the headline line: the CeAl-like cell (the default, the largest "
                         "single-GPU configuration) or the LiH-like cell (for its own counter profiles)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path "
              f"(asked for {args.gpus}); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1611_00731_amd as P
    import workloads as W
    from paper_1611_00731_amd import build as libbuild
    from workloads.potential import potential_at

    if libbuild.stale():
        log("warning: libpufe.so is older than its sources; rebuild before trusting these numbers")
    tune_cache = os.environ.get("PUFE_TUNE_CACHE")
    dev = torch.device("cuda", 0)
    prob = W.ceal_cell() if args.workload == "ceal" else W.lih_cell()
    log("setup", prob["name"])
    p = P.Problem(prob).setup()
    if not args.no_tune:
        log("autotune")
        t0 = time.perf_counter()
        P.pufe_tune(p.ctx, args.precision, tune_cache)
        log(f"autotune {time.perf_counter() - t0:.1f} s")
    sz = p.sizes
    xyz, w, qp_off = p.quadrature()
    V = potential_at(xyz.cpu(), prob).to(dev) if args.host_inputs else potential_at(xyz, prob)
    del xyz, w, qp_off
    lay = p.layout()
    _, _, leaf_off = p.leaves()
    nloc, nq, flops = element_work(prob, sz, lay, leaf_off, prob["quad"]["n"] ** 3)
    kpts = prob["kpts"]
    n_out = len(kpts)
    H = torch.empty((n_out, sz["nnz"], 2), dtype=torch.float64, device=dev)
    S = torch.empty_like(H)
    log(f"n_elem {sz['n_elem']} n_qp {sz['n_qp']} n_dof {sz['n_dof']} nnz {sz['nnz']} k-points {n_out}")
    ms_step, ms_instr, kern = time_assembly(P, p, V, kpts, args.precision, H, S, args.steps, args.warmup)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (instrumented {ms_instr:.3f})")
    contract_ms = kern["contract_ms"]
    alg_flops = float(flops.sum())
    achieved = alg_flops / (contract_ms * 1e-3) / 1e12
    value = sz["n_elem"] * n_out / (ms_step * 1e-3)
    tag = "contract_f64_ceal_cell" if args.workload == "ceal" else "contract_f64_lih_cell"
    traffic, = recorded(tag + "_hbm_traffic.md", "traffic_bytes_per_launch")
    busy, executed = recorded(tag + "_mfma_counters.md", "mfma_busy_frac", "mfma_executed_flops_per_launch")
    fp64 = args.precision == "fp64"
    out = {
        "metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64 else args.precision,
        "data": "synthetic",
        "config": {"workload": ("CeAl-like CsCl cell a=5.8 bohr, 12^3 triquadratic hexes, 8^3 Gauss + 3 octree "
                                "levels within 1 bohr, 4 k-points (time-reversal-reduced 2x2x2 MP), "
                                "H+S complex128, autotuned") if args.workload == "ceal" else
                               ("LiH-like rock-salt cell a=7.6 bohr, 8^3 triquadratic hexes, 6^3 Gauss + 2 octree "
                                "levels within 1 bohr, Gamma, H+S complex128, autotuned"),
                   "n_elem": sz["n_elem"], "n_qp": sz["n_qp"], "n_dof": sz["n_dof"],
                   "nnz": sz["nnz"], "kpoints": n_out, "precision": args.precision,
                   "nloc_min": int(nloc.min()), "nloc_max": int(nloc.max()), "nq_max": int(nq.max())},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[args.precision],
                     "traffic": traffic if fp64 else None,
                     "kernel": ("contract_f64_wide_kernel + contract_f64_kernel (the two launches of one "
                                "contraction, timed as one region)") if fp64 else "contract_split_kernel",
                     "kernel_ms": contract_ms, "alg_flops_per_launch": alg_flops,
                     "mfma_busy_frac": busy if fp64 else None,
                     "mfma_executed_flops_per_launch": executed if fp64 else None},
        "extra": {"ms_per_step_with_kernel_events": ms_instr,
                  "scatter_ms_per_assembly": kern["scatter_ms_per_assembly"],
                  "chunk_reduce_ms": kern["chunk_reduce_ms"],
                  "gflops_step": alg_flops / (ms_step * 1e-3) / 1e9,
                  "unique_contractions_per_s": sz["n_elem"] / (ms_step * 1e-3)},
    }
    if traffic is not None and fp64:
        gbs = traffic / (contract_ms * 1e-3) / 1e9
        out["roofline"]["hbm_gbs"] = gbs
        out["roofline"]["hbm_frac"] = gbs / HBM_PEAK_GBS
    # the paper's own figures, quoted as context (it gives no timings or hardware)
    out["paper_context"] = ("no timings, FLOP rates or hardware are published for this method; the paper's "
                            "figures are basis sizes: cubic PUFE needs about 12x (LiH) and 5x (CeAl) fewer "
                            "DOFs than plane waves at 1e-3 Ha/atom, 269 PUFE functions against 2398-4132 plane "
                            "waves in the LiH equation of state, and the overlap sparsity of its Table 1")
    if fp64 and not args.no_split:
        log("split-BF16 forms on the same inputs")
        sp = leg_ceal_split(P, p, V, kpts, alg_flops, H, S)
        for prec in sp:
            sp[prec]["speedup_vs_fp64_contraction"] = contract_ms / sp[prec]["contract_ms"]
        out["extra"]["split"] = sp
    del H, S
    p.close()
    do_eig = not (args.no_eig or args.host_inputs)
    if not args.no_rows and fp64:
        log("LiH-like cell leg")
        out["extra"]["lih_cell"] = leg_lih_cell(P, W, potential_at, 20, 3, tune_cache, do_eig)
        if do_eig:
            out["eig_err"] = out["extra"]["lih_cell"].pop("eig_err")
        log("batch leg (lattice sweep)")
        out["extra"]["batch_sweep"] = leg_batch(tune_cache)
        log("adjoint leg (64-atom supercell)")
        out["extra"]["adjoint"] = leg_backward()
        log("nonlocal leg (LiH-like cell with projectors)")
        out["extra"]["nonlocal"] = leg_nonlocal(P, W, potential_at)
        log("Bloch-periodic enrichment leg (LiH-like cell, 4 k-points)")
        out["extra"]["bloch"] = leg_bloch(P, W, potential_at)
        log("self-consistent field leg (LiH-like cell)")
        out["extra"]["scf"] = leg_scf(P, W, potential_at)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(prob, n_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
