"""CPU emulation of the split-BF16 contraction's limb arithmetic.

The split kernels form every product of the element contraction (eq.
disceig3d) from bf16 limbs of the FP64 operands: the first limb is the
operand rounded to FP32 and then to bf16 (round to nearest even), each
further limb the same rounding of the residual carried in FP32.  Two limbs
keep the products a0 b0 + a0 b1 + a1 b0 (bf16x3), three add a1 b1 + a0 b2 +
a2 b0 (bf16x6).  One MFMA sums 32 points of one operand component; every
component has an FP32 accumulator per 32-point stage, added into FP64 after
the stage.  Here that scheme is replayed in numpy on the weighted basis rows
of elements of the LiH-like cell (the oracle's basis values at the oracle's
points), each MFMA taken as the exact sum of its limb products rounded once
to FP32 (bf16 x bf16 products are exact in FP32), and compared with the same
contraction in FP64.

What it shows: three limbs keep the element matrices near 1e-8 relative;
two limbs leave errors of order 2e-6 in H and S, over the 1e-7 split target.
Most of that is a bias rather than rounding noise: the dropped product
a1 b1 is, for a = b (and for the strongly correlated neighbouring rows),
the square of one residual, positive at every point, so its error grows with
the number of points instead of averaging out (about 2^-18 / 3 of the
product each).  Keeping a1 b1 as a fourth product removes most of it, which
an estimate assuming independent errors per point would miss.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def bf16_rne(x32):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    u = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def limbs(x, nl):
    """bf16 limbs of FP64 values x as the kernels form them."""
    out = [bf16_rne(x.astype(np.float32))]
    r = (x - out[0].astype(np.float64)).astype(np.float32)
    for _ in range(1, nl):
        h = bf16_rne(r)
        out.append(h)
        r = (r - h).astype(np.float32)
    return out


PAIRS = {2: [(0, 1), (1, 0), (0, 0)], 3: [(2, 0), (0, 2), (1, 1), (0, 1), (1, 0), (0, 0)],
         # two limbs with the a1 b1 product kept (not a kernel form; isolates the bias)
         "2+11": [(1, 1), (0, 1), (1, 0), (0, 0)]}


def split_product(A, B, nl, stage=32):
    """sum_q A[a, q] B[b, q] with the kernels' limb scheme: FP32 per
    32-point stage (one rounding per MFMA, products in the kernels' order),
    FP64 across stages."""
    nlimb = 2 if nl == "2+11" else nl
    la, lb = limbs(A, nlimb), limbs(B, nlimb)
    n, K = A.shape
    out = np.zeros((n, n))
    for s in range(0, K, stage):
        acc = np.zeros((n, n), np.float32)
        for i, j in PAIRS[nl]:
            blk = la[i][:, s:s + stage].astype(np.float64) @ lb[j][:, s:s + stage].astype(np.float64).T
            acc = (acc.astype(np.float64) + blk).astype(np.float32)
        out += acc.astype(np.float64)
    return out


def element_rows(o, prob, quad, e):
    """Weighted rows of element e at the oracle's points: sqrt(w/2) grad phi
    (3 components), sqrt(w) phi, and V sqrt(w) phi."""
    lev, ijk, loff = o.leaves()
    n = prob["quad"]["n"]
    g, _ = np.polynomial.legendre.leggauss(n)
    xyz, w, qoff = quad
    xs, ws = xyz[qoff[e]:qoff[e + 1]], w[qoff[e]:qoff[e + 1]]
    V = oracle.potential_np(xs, prob)
    pts = []
    for k in range(loff[e], loff[e + 1]):
        h = 2.0 / 2 ** lev[k]
        for a3 in range(n):
            for a2 in range(n):
                for a1 in range(n):
                    pts.append([-1 + (ijk[k][d] + 0.5) * h + 0.5 * h * g[a] for d, a in enumerate((a1, a2, a3))])
    vals, grads = zip(*[o.basis_at(e, xi) for xi in pts])
    phi = np.array(vals).T                       # n_loc x n_q
    grad = np.array(grads).transpose(1, 2, 0)    # n_loc x 3 x n_q
    s2, sw = np.sqrt(ws / 2), np.sqrt(ws)
    G = grad * s2
    U = phi * sw
    return G, U, V * U


def contract(G, U, VU, nl=None):
    f = (lambda A, B: A @ B.T) if nl is None else (lambda A, B: split_product(A, B, nl))
    H = f(G[:, 0], G[:, 0]) + f(G[:, 1], G[:, 1]) + f(G[:, 2], G[:, 2]) + f(VU, U)
    S = f(U, U)
    return H, S


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def lih():
    prob = W.lih_cell()
    o = oracle.Oracle(prob)
    _, _, loff = o.leaves()
    nl = np.diff(loff)
    refined = int(np.nonzero(nl > 1)[0][0])
    plain = int(np.nonzero(nl == 1)[0][0])
    return prob, o, o.quadrature(), [refined, plain]


def test_limbs_reconstruct_operands():
    x = np.random.default_rng(0).normal(size=10000) * 10.0 ** np.random.default_rng(1).uniform(-3, 3, 10000)
    for nl, bits in ((2, 16), (3, 24)):
        r = sum(l.astype(np.float64) for l in limbs(x, nl))
        # each bf16 limb carries 8 significant bits
        assert np.max(np.abs(r - x) / np.abs(x)) < 2.0 ** -(bits - 1)


def test_split_scheme_errors_on_lih_cell_elements(lih):
    prob, o, quad, elems = lih
    for e in elems:
        G, U, VU = element_rows(o, prob, quad, e)
        H, S = contract(G, U, VU)
        H6, S6 = contract(G, U, VU, 3)
        H3, S3 = contract(G, U, VU, 2)
        H4, S4 = contract(G, U, VU, "2+11")
        e6 = max(rel(H6, H), rel(S6, S))
        e3h, e3s = rel(H3, H), rel(S3, S)
        e4 = max(rel(H4, H), rel(S4, S))
        print(f"element {e} n_q {U.shape[1]} n_loc {U.shape[0]}: bf16x6 {e6:.2e}; bf16x3 H {e3h:.2e} "
              f"S {e3s:.2e}; two limbs with a1 b1 kept {e4:.2e}")
        assert e6 < 1e-7                       # three limbs meet the split target
        assert 1e-7 < min(e3h, e3s) < 1e-5     # two limbs cannot
        assert e4 < 0.6 * max(e3h, e3s)        # the dropped a1 b1 is the larger part of the error
