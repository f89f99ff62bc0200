"""Python binding of libpufe (the MI355X PUFE assembly library).

Thin ctypes layer over the C ABI in include/pufe.h: the functions below carry
the same names as the C entry points and only marshal arguments.  Device
buffers are torch tensors on the context's device; every step of the path
runs in the library's HIP kernels.  Importing this package fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpufe.so")

PUFE_OK = 0
ERRORS = {-1: "PUFE_ERR_INVALID_ARG", -2: "PUFE_ERR_UNSUPPORTED", -3: "PUFE_ERR_OOM",
          -4: "PUFE_ERR_HIP", -5: "PUFE_ERR_STATE"}
PREC = {"fp64": 0, "bf16x3": 1, "bf16x6": 2}
OUT = {"c128": 0, "c64": 1, "f64": 2}
QUAD_MODE = {"geom": 0, "error": 1}
ENR_PHASE = {"periodic": 0, "bloch": 1}

EXPORTS = ["pufe_error_string", "pufe_last_error_message", "pufe_create", "pufe_destroy",
           "pufe_set_problem", "pufe_setup", "pufe_query", "pufe_get_layout",
           "pufe_get_quadrature", "pufe_get_leaves", "pufe_assemble", "pufe_element_matrices",
           "pufe_assemble_backward", "pufe_bsr_to_dense", "pufe_enable_timing",
           "pufe_kernel_times", "pufe_set_positions", "pufe_batch_create", "pufe_batch_assemble",
           "pufe_batch_destroy", "pufe_batch_last_error_message", "pufe_tune", "pufe_assemble_noalloc", "pufe_set_rule", "pufe_set_projectors",
           "pufe_set_enrichment_phase", "pufe_fe_load", "pufe_fe_eval", "pufe_hartree", "pufe_lda_xc"]


class PufeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class pufe_enrichment(C.Structure):
    _fields_ = [("species", C.c_int), ("l", C.c_int), ("radial_kind", C.c_int),
                ("a", C.c_double), ("rc", C.c_double), ("re", C.c_double),
                ("radial", C.POINTER(C.c_double)), ("n_radial", C.c_int)]


class pufe_projector(C.Structure):
    _fields_ = [("species", C.c_int), ("l", C.c_int), ("a", C.c_double), ("rc", C.c_double), ("h", C.c_double)]


class pufe_quad(C.Structure):
    _fields_ = [("n_gauss", C.c_int), ("n_ref", C.c_int), ("max_level", C.c_int),
                ("mode", C.c_int), ("dist", C.c_double), ("tol", C.c_double)]


class pufe_sizes(C.Structure):
    _fields_ = [("n_elem", C.c_int64), ("n_vertex", C.c_int64), ("n_dof", C.c_int64),
                ("n_fe_dof", C.c_int64), ("n_enr_dof", C.c_int64), ("nnzb", C.c_int64),
                ("nnz", C.c_int64), ("n_qp", C.c_int64), ("n_leaves", C.c_int64),
                ("max_nloc", C.c_int32), ("n_colors", C.c_int32), ("n_atoms", C.c_int32),
                ("n_fe_slots", C.c_int32)]


def _load():
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that runtime instead of a second copy
    # (two runtimes in one process do not share devices, streams or memory)
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpufe.so is not built ({LIB_PATH}); run python -m paper_1611_00731_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i64p, i32p, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    sig = {
        "pufe_error_string": ([C.c_int], C.c_char_p),
        "pufe_last_error_message": ([vp], C.c_char_p),
        "pufe_create": ([C.POINTER(vp), C.c_int], C.c_int),
        "pufe_destroy": ([vp], C.c_int),
        "pufe_set_problem": ([vp, dp, C.POINTER(C.c_int), C.c_int, C.c_int, dp, C.POINTER(C.c_int),
                              C.c_int, C.POINTER(pufe_enrichment), C.POINTER(pufe_quad)], C.c_int),
        "pufe_setup": ([vp, vp], C.c_int),
        "pufe_query": ([vp, C.POINTER(pufe_sizes)], C.c_int),
        "pufe_get_layout": ([vp, i64p, i64p, i32p, i64p], C.c_int),
        "pufe_get_quadrature": ([vp, vp, vp, vp, vp], C.c_int),
        "pufe_get_leaves": ([vp, i32p, i32p, i64p], C.c_int),
        "pufe_assemble": ([vp, vp, dp, C.c_int, C.c_int, C.c_int, vp, vp, vp], C.c_int),
        "pufe_assemble_noalloc": ([vp, vp, dp, C.c_int, C.c_int, C.c_int, vp, vp, vp], C.c_int),
        "pufe_set_rule": ([vp, C.c_int64, i32p, i32p, i64p, vp], C.c_int),
        "pufe_set_projectors": ([vp, C.c_int, C.POINTER(pufe_projector)], C.c_int),
        "pufe_set_enrichment_phase": ([vp, C.c_int], C.c_int),
        "pufe_fe_load": ([vp, vp, vp, vp], C.c_int),
        "pufe_fe_eval": ([vp, vp, vp, vp], C.c_int),
        "pufe_hartree": ([vp, vp, vp, vp, C.c_double, C.c_int, C.POINTER(C.c_int), dp, vp], C.c_int),
        "pufe_lda_xc": ([C.c_int64, vp, vp, vp, vp], C.c_int),
        "pufe_element_matrices": ([vp, C.c_int64, vp, C.c_int, vp, vp, i32p, vp], C.c_int),
        "pufe_assemble_backward": ([vp, vp, dp, vp, vp, C.c_int, vp, vp, vp], C.c_int),
        "pufe_bsr_to_dense": ([vp, vp, C.c_int, vp, vp], C.c_int),
        "pufe_enable_timing": ([vp, C.c_int], C.c_int),
        "pufe_kernel_times": ([vp, dp, i64p, C.c_int], C.c_int),
        "pufe_set_positions": ([vp, dp], C.c_int),
        "pufe_batch_create": ([C.POINTER(vp), C.POINTER(vp), C.c_int], C.c_int),
        "pufe_batch_assemble": ([vp, C.POINTER(vp), dp, C.c_int, C.c_int, C.c_int, C.POINTER(vp),
                                 C.POINTER(vp), vp], C.c_int),
        "pufe_batch_destroy": ([vp], C.c_int),
        "pufe_batch_last_error_message": ([vp], C.c_char_p),
        "pufe_tune": ([vp, C.c_int, C.c_char_p], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def _check(ctx, rc):
    if rc != PUFE_OK:
        msg = lib.pufe_last_error_message(ctx).decode() if ctx else ""
        raise PufeError(rc, msg)


def _ptr(t):
    """Device (or host) address of a torch tensor, None for None."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C names

def pufe_create(device: int = 0):
    h = C.c_void_p()
    _check(None, lib.pufe_create(C.byref(h), device))
    return h


def pufe_destroy(ctx):
    _check(None, lib.pufe_destroy(ctx))


def pufe_set_problem(ctx, lattice, mesh, fe_order, pos, species, enrichments, quad):
    lat = (C.c_double * 9)(*np.asarray(lattice, float).reshape(9))
    msh = (C.c_int * 3)(*[int(m) for m in mesh])
    pos = np.ascontiguousarray(np.asarray(pos, np.float64).reshape(-1))
    spc = np.ascontiguousarray(np.asarray(species, np.int32).reshape(-1))
    n_atoms = spc.size
    enr = (pufe_enrichment * max(1, len(enrichments)))()
    keep = []   # sample arrays stay alive until the call has copied them
    for i, e in enumerate(enrichments):
        tab = e.get("radial")
        kind = int(e.get("radial_kind", 0 if tab is None else 1))
        ptr, n = None, 0
        if tab is not None:
            arr = np.ascontiguousarray(np.asarray(tab, np.float64).reshape(-1))
            keep.append(arr)
            ptr, n = arr.ctypes.data_as(C.POINTER(C.c_double)), arr.size
        enr[i] = pufe_enrichment(int(e["species"]), int(e["l"]), kind,
                                 float(e.get("a", 1.0)), float(e["rc"]), float(e["re"]), ptr, n)
    q = pufe_quad(int(quad["n"]), int(quad.get("n_ref", quad["n"] + 1)), int(quad["levels"]),
                  QUAD_MODE[quad.get("mode", "geom")], float(quad.get("dist", 0.0)),
                  float(quad.get("tol", 1e-6)))
    _check(ctx, lib.pufe_set_problem(
        ctx, lat, msh, int(fe_order), n_atoms,
        pos.ctypes.data_as(C.POINTER(C.c_double)), spc.ctypes.data_as(C.POINTER(C.c_int)),
        len(enrichments), enr, C.byref(q)))


def pufe_set_projectors(ctx, projectors):
    arr = (pufe_projector * max(1, len(projectors)))()
    for i, q in enumerate(projectors):
        arr[i] = pufe_projector(int(q["species"]), int(q["l"]), float(q["a"]), float(q["rc"]), float(q["h"]))
    _check(ctx, lib.pufe_set_projectors(ctx, len(projectors), arr))


def pufe_set_enrichment_phase(ctx, form):
    """form: "periodic" (f(R) = 1) or "bloch" (f(R) = exp(i k.R)) of eq. Psi."""
    _check(ctx, lib.pufe_set_enrichment_phase(ctx, ENR_PHASE[form]))


def pufe_setup(ctx, stream=None):
    _check(ctx, lib.pufe_setup(ctx, _stream(stream)))


def pufe_query(ctx) -> dict:
    s = pufe_sizes()
    _check(ctx, lib.pufe_query(ctx, C.byref(s)))
    return {f: getattr(s, f) for f, _ in pufe_sizes._fields_}


def pufe_get_layout(ctx):
    sz = pufe_query(ctx)
    dof = np.zeros(sz["n_vertex"] + 1, np.int64)
    rp = np.zeros(sz["n_vertex"] + 1, np.int64)
    bc = np.zeros(max(1, sz["nnzb"]), np.int32)
    bo = np.zeros(sz["nnzb"] + 1, np.int64)
    i64p, i32p = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    _check(ctx, lib.pufe_get_layout(ctx, dof.ctypes.data_as(i64p), rp.ctypes.data_as(i64p),
                                    bc.ctypes.data_as(i32p), bo.ctypes.data_as(i64p)))
    return {"dof_offset": dof, "brow_ptr": rp, "bcol": bc[:sz["nnzb"]], "bval_offset": bo}


def pufe_get_quadrature(ctx, xyz=None, w=None, elem_qp_offset=None, stream=None):
    _check(ctx, lib.pufe_get_quadrature(ctx, _ptr(xyz), _ptr(w), _ptr(elem_qp_offset), _stream(stream)))


def pufe_get_leaves(ctx):
    sz = pufe_query(ctx)
    n = sz["n_leaves"]
    lev = np.zeros(max(n, 1), np.int32)
    ijk = np.zeros(3 * max(n, 1), np.int32)
    off = np.zeros(sz["n_elem"] + 1, np.int64)
    i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    _check(ctx, lib.pufe_get_leaves(ctx, lev.ctypes.data_as(i32p), ijk.ctypes.data_as(i32p),
                                    off.ctypes.data_as(i64p)))
    return lev[:n], ijk[:3 * n].reshape(-1, 3), off


def pufe_set_rule(ctx, level, ijk, elem_leaf_offset, stream=None):
    lev = np.ascontiguousarray(np.asarray(level, np.int32))
    c = np.ascontiguousarray(np.asarray(ijk, np.int32).reshape(-1))
    off = np.ascontiguousarray(np.asarray(elem_leaf_offset, np.int64))
    i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    _check(ctx, lib.pufe_set_rule(ctx, lev.size, lev.ctypes.data_as(i32p), c.ctypes.data_as(i32p),
                                  off.ctypes.data_as(i64p), _stream(stream)))


def pufe_assemble(ctx, V, kpts, precision, out_dtype, H, S=None, stream=None):
    k = np.ascontiguousarray(np.asarray(kpts, np.float64).reshape(-1, 3))
    _check(ctx, lib.pufe_assemble(ctx, _ptr(V), k.ctypes.data_as(C.POINTER(C.c_double)), k.shape[0],
                                  PREC[precision] if isinstance(precision, str) else int(precision),
                                  OUT[out_dtype] if isinstance(out_dtype, str) else int(out_dtype),
                                  _ptr(H), _ptr(S), _stream(stream)))


def pufe_assemble_noalloc(ctx, V, kpts, precision, out_dtype, H, S=None, stream=None):
    k = np.ascontiguousarray(np.asarray(kpts, np.float64).reshape(-1, 3))
    _check(ctx, lib.pufe_assemble_noalloc(ctx, _ptr(V), k.ctypes.data_as(C.POINTER(C.c_double)), k.shape[0],
                                          PREC[precision] if isinstance(precision, str) else int(precision),
                                          OUT[out_dtype] if isinstance(out_dtype, str) else int(out_dtype),
                                          _ptr(H), _ptr(S), _stream(stream)))


def pufe_element_matrices(ctx, elem, V, precision, He, Se, stream=None):
    n = C.c_int32()
    _check(ctx, lib.pufe_element_matrices(ctx, int(elem), _ptr(V),
                                          PREC[precision] if isinstance(precision, str) else int(precision),
                                          _ptr(He), _ptr(Se), C.byref(n), _stream(stream)))
    return n.value


def pufe_assemble_backward(ctx, V, kpt, P, Q, precision, dLdV, dLdR, stream=None):
    k = (C.c_double * 3)(*[float(x) for x in kpt])
    _check(ctx, lib.pufe_assemble_backward(ctx, _ptr(V), k, _ptr(P), _ptr(Q),
                                           PREC[precision] if isinstance(precision, str) else int(precision),
                                           _ptr(dLdV), _ptr(dLdR), _stream(stream)))


def pufe_bsr_to_dense(ctx, bsr, dtype, dense, stream=None):
    _check(ctx, lib.pufe_bsr_to_dense(ctx, _ptr(bsr), OUT[dtype] if isinstance(dtype, str) else int(dtype),
                                      _ptr(dense), _stream(stream)))


def pufe_set_positions(ctx, pos):
    p = np.ascontiguousarray(np.asarray(pos, np.float64).reshape(-1))
    _check(ctx, lib.pufe_set_positions(ctx, p.ctypes.data_as(C.POINTER(C.c_double))))


def pufe_fe_load(ctx, f, b, stream=None):
    _check(ctx, lib.pufe_fe_load(ctx, _ptr(f), _ptr(b), _stream(stream)))


def pufe_fe_eval(ctx, u, out, stream=None):
    _check(ctx, lib.pufe_fe_eval(ctx, _ptr(u), _ptr(out), _stream(stream)))


def pufe_hartree(ctx, n, vh, v=None, tol=1e-13, max_iter=5000, stream=None):
    """Returns (CG iterations, final relative residual)."""
    it = C.c_int(0)
    res = C.c_double(0.0)
    _check(ctx, lib.pufe_hartree(ctx, _ptr(n), _ptr(vh), _ptr(v), float(tol), int(max_iter), C.byref(it),
                                 C.byref(res), _stream(stream)))
    return it.value, res.value


def pufe_lda_xc(rho, vxc, exc=None, stream=None):
    rc = lib.pufe_lda_xc(rho.numel(), _ptr(rho), _ptr(vxc), _ptr(exc), _stream(stream))
    if rc != PUFE_OK:
        raise PufeError(rc, "pufe_lda_xc")


def pufe_enable_timing(ctx, on=True):
    _check(ctx, lib.pufe_enable_timing(ctx, 1 if on else 0))


def pufe_kernel_times(ctx, reset=True):
    ms = (C.c_double * 5)()
    cnt = (C.c_int64 * 5)()
    _check(ctx, lib.pufe_kernel_times(ctx, ms, cnt, 1 if reset else 0))
    return list(ms), list(cnt)


def pufe_tune(ctx, precision="fp64", cache_path=None):
    _check(ctx, lib.pufe_tune(ctx, PREC[precision] if isinstance(precision, str) else int(precision),
                              None if cache_path is None else str(cache_path).encode()))


def pufe_batch_create(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    h = C.c_void_p()
    rc = lib.pufe_batch_create(C.byref(h), arr, len(ctxs))
    if rc != PUFE_OK:
        raise PufeError(rc, "batch creation")
    return h


def pufe_batch_destroy(b):
    _check(None, lib.pufe_batch_destroy(b))


def pufe_batch_assemble(b, Vs, kpts, precision, out_dtype, Hs, Ss=None, stream=None):
    n = len(Vs)
    k = np.ascontiguousarray(np.asarray(kpts, np.float64).reshape(-1, 3))
    v = (C.c_void_p * n)(*[t.data_ptr() for t in Vs])
    h = (C.c_void_p * n)(*[t.data_ptr() for t in Hs])
    s = None if Ss is None else (C.c_void_p * n)(*[t.data_ptr() for t in Ss])
    rc = lib.pufe_batch_assemble(b, v, k.ctypes.data_as(C.POINTER(C.c_double)), k.shape[0],
                                 PREC[precision] if isinstance(precision, str) else int(precision),
                                 OUT[out_dtype] if isinstance(out_dtype, str) else int(out_dtype),
                                 h, s, _stream(stream))
    if rc != PUFE_OK:
        raise PufeError(rc, lib.pufe_batch_last_error_message(b).decode())


# --------------------------------------------------------- convenience layer

class Problem:
    """A problem dictionary (see the `workloads` package) bound to a context."""

    def __init__(self, prob: dict, device: int = 0):
        self.prob = prob
        self.device = device
        self.ctx = pufe_create(device)
        pufe_set_problem(self.ctx, prob["lattice"], prob["mesh"], prob["fe_order"], prob["atoms"],
                         prob["species"], prob["enrichments"], prob["quad"])
        if prob.get("projectors"):
            pufe_set_projectors(self.ctx, prob["projectors"])
        if prob.get("enrichment_phase", "periodic") != "periodic":
            pufe_set_enrichment_phase(self.ctx, prob["enrichment_phase"])
        self.sizes = pufe_query(self.ctx)
        self._ready = False

    def close(self):
        if getattr(self, "ctx", None):
            pufe_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, stream=None):
        pufe_setup(self.ctx, stream)
        self.sizes = pufe_query(self.ctx)
        self._ready = True
        return self

    def layout(self):
        return pufe_get_layout(self.ctx)

    def set_rule(self, level, ijk, elem_leaf_offset):
        pufe_set_rule(self.ctx, level, ijk, elem_leaf_offset)
        self.sizes = pufe_query(self.ctx)

    def leaves(self):
        return pufe_get_leaves(self.ctx)

    def quadrature(self):
        import torch
        dev = torch.device("cuda", self.device)
        n = self.sizes["n_qp"]
        xyz = torch.empty((n, 3), dtype=torch.float64, device=dev)
        w = torch.empty(n, dtype=torch.float64, device=dev)
        off = torch.empty(self.sizes["n_elem"] + 1, dtype=torch.int64, device=dev)
        pufe_get_quadrature(self.ctx, xyz, w, off)
        return xyz, w, off

    def assemble(self, V, kpts=((0.0, 0.0, 0.0),), precision="fp64", out_dtype="c128", with_S=True):
        import torch
        nk = len(kpts)
        nnz = self.sizes["nnz"]
        if out_dtype == "c128":
            shape, dt = (nk, nnz, 2), torch.float64
        elif out_dtype == "c64":
            shape, dt = (nk, nnz, 2), torch.float32
        else:
            shape, dt = (nk, nnz), torch.float64
        H = torch.empty(shape, dtype=dt, device=V.device)
        S = torch.empty(shape, dtype=dt, device=V.device) if with_S else None
        pufe_assemble(self.ctx, V, kpts, precision, out_dtype, H, S)
        return H, S

    def element_matrices(self, elem, V, precision="fp64"):
        import torch
        m = self.sizes["max_nloc"]
        He = torch.zeros((m, m), dtype=torch.float64, device=V.device)
        Se = torch.zeros((m, m), dtype=torch.float64, device=V.device)
        n = pufe_element_matrices(self.ctx, elem, V, precision, He, Se)
        return He.view(-1)[:n * n].view(n, n), Se.view(-1)[:n * n].view(n, n)

    def set_positions(self, pos):
        pufe_set_positions(self.ctx, pos)

    def backward(self, V, kpt, P=None, Q=None, want_dV=True, want_dR=True, precision="fp64"):
        """dL/dV (n_qp) and dL/dR (n_atoms x 3) for L = Re<P, H> + Re<Q, S>;
        P and Q are BSR value arrays (complex128 or (nnz, 2) float64)."""
        import torch
        dV = torch.empty(self.sizes["n_qp"], dtype=torch.float64, device=V.device) if want_dV else None
        dR = torch.empty((self.sizes["n_atoms"], 3), dtype=torch.float64, device=V.device) if want_dR else None
        pufe_assemble_backward(self.ctx, V, kpt, None if P is None else P.contiguous(),
                               None if Q is None else Q.contiguous(), precision, dV, dR)
        return dV, dR

    # self-consistent field pieces: vectors of the classical FE space have
    # n_vertex * n_fe_slots entries
    def fe_load(self, f):
        import torch
        b = torch.empty(self.sizes["n_vertex"] * self.sizes["n_fe_slots"], dtype=torch.float64, device=f.device)
        pufe_fe_load(self.ctx, f.contiguous(), b)
        return b

    def fe_eval(self, u):
        import torch
        out = torch.empty(self.sizes["n_qp"], dtype=torch.float64, device=u.device)
        pufe_fe_eval(self.ctx, u.contiguous(), out)
        return out

    def hartree(self, n, tol=1e-13, max_iter=5000):
        """(V_H at the points, its FE coefficients, CG iterations, relative residual)."""
        import torch
        vh = torch.empty(self.sizes["n_qp"], dtype=torch.float64, device=n.device)
        v = torch.empty(self.sizes["n_vertex"] * self.sizes["n_fe_slots"], dtype=torch.float64, device=n.device)
        it, res = pufe_hartree(self.ctx, n.contiguous(), vh, v, tol, max_iter)
        return vh, v, it, res

    def to_dense(self, bsr, dtype="c128"):
        import torch
        n = self.sizes["n_dof"]
        D = torch.empty((n, n, 2), dtype=torch.float64, device=bsr.device)
        pufe_bsr_to_dense(self.ctx, bsr.contiguous(), dtype, D)
        return torch.view_as_complex(D)


class Batch:
    """Several set-up problems assembled by one persistent, graph-captured launch."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.h = pufe_batch_create([p.ctx for p in self.problems])

    def close(self):
        if getattr(self, "h", None):
            pufe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, nk, out_dtype="c128", device=None):
        import torch
        dt = torch.float32 if out_dtype == "c64" else torch.float64
        last = () if out_dtype == "f64" else (2,)
        Hs = [torch.empty((nk, p.sizes["nnz"]) + last, dtype=dt, device=device) for p in self.problems]
        Ss = [torch.empty_like(h) for h in Hs]
        return Hs, Ss

    def assemble(self, Vs, kpts, Hs, Ss=None, precision="fp64", out_dtype="c128"):
        pufe_batch_assemble(self.h, Vs, kpts, precision, out_dtype, Hs, Ss)


def _make_autograd():
    import torch

    class PUFEAssemble(torch.autograd.Function):
        """H, S = PUFEAssemble.apply(problem, V, R, kpt): complex128 BSR values of
        one k-point as functions of the potential V at the quadrature points and
        of the enrichment centres R (n_atoms x 3; rule and enriched sets fixed).
        The backward pass calls the adjoint kernels; for a real loss L the
        incoming gradients are P = dL/dH and Q = dL/dS in torch's convention,
        i.e. L = Re<P, H> + Re<Q, S> to first order."""

        @staticmethod
        def forward(ctx, problem, V, R, kpt):
            problem.set_positions(R.detach().cpu().numpy())
            nnz = problem.sizes["nnz"]
            H = torch.empty(nnz, dtype=torch.complex128, device=V.device)
            S = torch.empty(nnz, dtype=torch.complex128, device=V.device)
            pufe_assemble(problem.ctx, V.detach().contiguous(), [kpt], "fp64", "c128", H, S)
            ctx.problem = problem
            ctx.kpt = tuple(float(k) for k in kpt)
            ctx.R = R.detach().cpu().numpy()
            ctx.R_device = R.device
            ctx.save_for_backward(V)
            return H, S

        @staticmethod
        def backward(ctx, gH, gS):
            (V,) = ctx.saved_tensors
            ctx.problem.set_positions(ctx.R)
            dV, dR = ctx.problem.backward(V.detach().contiguous(), ctx.kpt, gH, gS)
            return None, dV, dR.to(ctx.R_device), None

    return PUFEAssemble


class _Lazy:
    cls = None


def PUFEAssemble():
    if _Lazy.cls is None:
        _Lazy.cls = _make_autograd()
    return _Lazy.cls


def _tril_inverse(L, base=256):
    """Inverse of a lower-triangular matrix by 2x2 block recursion: GEMMs
    plus triangular solves of at most `base` columns at the leaves."""
    import torch
    n = L.shape[0]
    if n <= base:
        eye = torch.eye(n, dtype=L.dtype, device=L.device)
        return torch.linalg.solve_triangular(L, eye, upper=False)
    h = n // 2
    Ai = _tril_inverse(L[:h, :h], base)
    Ci = _tril_inverse(L[h:, h:].contiguous(), base)
    out = torch.zeros_like(L)
    out[:h, :h] = Ai
    out[h:, h:] = Ci
    out[h:, :h] = -(Ci @ (L[h:, :h] @ Ai))
    return out


def eigh(H, S):
    """All eigenpairs of H c = eps S c (eq. disceig3d) on the device in FP64,
    by the reduction of eig: eigenvalues ascending, eigenvectors as columns,
    normalised so that c^H S c = 1.  A reduced matrix with no imaginary part
    (Gamma) goes to the real symmetric solver: the device's complex Hermitian
    solver has returned non-finite eigenvectors for such matrices of a few
    thousand rows.  Non-finite results raise."""
    import torch
    Lc = torch.linalg.cholesky(0.5 * (S + S.mH))
    Li = _tril_inverse(Lc)
    A = Li @ H @ Li.mH
    A = 0.5 * (A + A.mH)
    if A.is_complex() and int(torch.count_nonzero(A.imag)) == 0:
        e, Yr = torch.linalg.eigh(A.real.contiguous())
        Y = Yr.to(A.dtype)
    else:
        e, Y = torch.linalg.eigh(A)
    Yv = torch.view_as_real(Y) if Y.is_complex() else Y
    if not bool(torch.isfinite(Yv).all()) or not bool(torch.isfinite(e).all()):
        raise RuntimeError("the dense eigensolver returned non-finite eigenpairs")
    return e, Li.mH @ Y


def eig(H, S, m):
    """Lowest m eigenvalues of H c = eps S c (eq. disceig3d) on the device in
    FP64: S = L L^H (Cholesky), eigenvalues of the Hermitian L^-1 H L^-H.
    L^-1 is formed by block recursion (GEMMs and small triangular solves),
    since one large triangular solve needs more library workspace than is
    available at a few thousand DOFs."""
    import torch
    Lc = torch.linalg.cholesky(0.5 * (S + S.mH))
    Li = _tril_inverse(Lc)
    A = Li @ H @ Li.mH
    A = 0.5 * (A + A.mH)
    return torch.linalg.eigvalsh(A)[:m]
