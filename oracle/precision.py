"""Emulation of the lower-precision storage tiers (TEST INFRASTRUCTURE ONLY).

The paper's product (Sec. IV.B) is written for one precision.  The tiers store
the same blocks in fewer bits and accumulate in float32; this module computes,
step by step, what such a product yields, so that a device tier can be judged
against the FP64 oracle with a predicted error.

FP32 tier
    Every stored block entry (near blocks, couplings, leaf bases, transfers) is
    rounded to complex64, as are chi, x and sigma k^2 V.  Each step of Sec. IV.B
    (forward transformation, upward pass, coupling multiplication, downward
    pass, backward transformation plus the inadmissible blocks) runs with
    complex64 operands and float32 accumulators; the coefficient vectors
    x^ and y^ are held in complex64 between the steps.

BF16 hi+lo tier ("bf16x3")
    Each float32 real part v is split into hi = bf16(v) and lo = bf16(v - hi)
    (round to nearest even); a product a*b is formed from the three terms
    hi_a hi_b + hi_a lo_b + lo_a hi_b (lo_a lo_b is dropped), the products being
    exact in float32 and their sums float32.  Both operands of every block
    product are split: the stored block, and the vector it multiplies, which is
    chi . x for the forward transformation and the inadmissible blocks, and the
    float32 coefficient vector x^ or y^ of the previous step otherwise.  So the
    coefficients are re-split after every step that produces them: after the
    forward transformation and each level of the upward pass (x^), after the
    coupling multiplication and each level of the downward pass (y^).  The
    downward pass adds T_c y^_p (formed in float32) to the coupling result y^_c
    already held in float32.  At each leaf, the inadmissible blocks and the leaf
    basis term V_t y^_t are summed in one float32 accumulator.

bf16 rounding is written out on the float32 bit pattern: add 0x7fff plus the
lowest kept bit, then clear the low 16 bits.

Pins (tests/test_precision_oracle.py): closed forms on a hand-built seven-cluster
description for the rounding of each block array and of x, for the dropped lo*lo
term and for each re-split; exact agreement with the FP64 oracle when every value
and partial sum is representable; planted mistakes that must break those pins.
"""

from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = ~np.isfinite(f)
    out = np.where(nan, f, out)
    return out.reshape(np.shape(x))


def split_bf16(z: np.ndarray):
    """(hi, lo) complex64 arrays with bf16-representable parts, hi + lo ~= z.

    z is first rounded to complex64 (the tier's float32 value), then each part
    is split."""
    re = np.asarray(np.real(z), np.float32)
    im = np.asarray(np.imag(z), np.float32)
    hr, hm = bf16_round(re), bf16_round(im)
    lr, lm = bf16_round(re - hr), bf16_round(im - hm)
    hi = np.empty(np.shape(re), np.complex64)
    lo = np.empty(np.shape(re), np.complex64)
    hi.real, hi.imag = hr, hm
    lo.real, lo.imag = lr, lm
    return hi, lo


# ------------------------------------------------------------------ operands
class _Fp32Operand:
    """A complex64 operand of the FP32 tier."""

    def __init__(self, v):
        self.v = np.asarray(v).astype(np.complex64)


class _SplitOperand:
    """The hi and lo parts of a BF16 tier operand."""

    def __init__(self, v):
        self.hi, self.lo = split_bf16(np.asarray(v))


def _mul_fp32(a: _Fp32Operand, b: _Fp32Operand) -> np.ndarray:
    return (a.v @ b.v).astype(np.complex64)


def _mul_bf16x3(a: _SplitOperand, b: _SplitOperand) -> np.ndarray:
    # each partial product of bf16 parts is exact in float32; the sums are float32
    p = a.hi @ b.hi
    p = p + a.hi @ b.lo
    p = p + a.lo @ b.hi
    return p.astype(np.complex64)


_OPERAND = {"fp32": _Fp32Operand, "bf16x3": _SplitOperand}
_MUL = {"fp32": _mul_fp32, "bf16x3": _mul_bf16x3}


def _block_operand(tier: str, which: str, B: np.ndarray):
    """A stored block (which: near, coupling, basis, transfer) as the tier holds it."""
    return _OPERAND[tier](B)


def _vector_operand(tier: str, u: np.ndarray):
    """The tree-ordered input chi . x (complex64) of one leaf."""
    return _OPERAND[tier](u)


def _coef_operand(tier: str, c: np.ndarray):
    """A float32 coefficient vector x^ or y^ used as the operand of the next step."""
    return _OPERAND[tier](c)


# ------------------------------------------------------------------ blocks
def _block(flat, off, rows, cols):
    """Column-major rows x cols block at element offset off."""
    return np.asarray(flat[off:off + rows * cols]).reshape(cols, rows).T


def _apply_tier(d, U32: np.ndarray, tier: str) -> np.ndarray:
    """y = G u in the tier, for u (n_vox, ncol) complex64 in tree order."""
    mul = _MUL[tier]
    nc = int(d.level.shape[0])
    depth = int(d.level.max())
    ncol = U32.shape[1]
    size = lambda c: int(d.end[c] - d.begin[c])
    rank = lambda c: int(d.rank[c])

    def basis(c):            # V_c, #c x k_c
        return _block(d.basis, int(d.basis_off[c]), size(c), rank(c))

    def transfer(c):         # T_c, k_c x k_parent
        return _block(d.transfer, int(d.transfer_off[c]), rank(c), rank(int(d.parent[c])))

    Uop = {c: _vector_operand(tier, U32[d.begin[c]:d.end[c]]) for c in range(nc) if d.nchild[c] == 0}
    zero = lambda k: np.zeros((k, ncol), np.complex64)

    # forward transformation at the leaves: x^_t = V_t^T u_t
    xh = {}
    for c in range(nc):
        if d.nchild[c] == 0 and rank(c) > 0:
            xh[c] = mul(_block_operand(tier, "basis", basis(c).T), Uop[c])
    # upward pass, deepest parents first: x^_p = sum_c T_c^T x^_c, each x^_c re-split
    for lev in range(depth - 1, -1, -1):
        for p in np.nonzero(d.level == lev)[0]:
            if d.nchild[p] == 0 or rank(p) == 0:
                continue
            acc = zero(rank(p))
            for ch in range(int(d.first_child[p]), int(d.first_child[p] + d.nchild[p])):
                if rank(ch) > 0:
                    acc = (acc + mul(_block_operand(tier, "transfer", transfer(ch).T),
                                     _coef_operand(tier, xh[ch]))).astype(np.complex64)
            xh[int(p)] = acc
    # coupling multiplication: y^_t = sum_s S_ts x^_s
    yh = {c: zero(rank(c)) for c in range(nc) if rank(c) > 0}
    for i in range(d.far_t.shape[0]):
        t, s = int(d.far_t[i]), int(d.far_s[i])
        S = _block(d.coupling, int(d.far_off[i]), rank(t), rank(s))
        yh[t] = (yh[t] + mul(_block_operand(tier, "coupling", S), _coef_operand(tier, xh[s]))).astype(np.complex64)
    # downward pass, top children first: y^_c += T_c y^_p, y^_p re-split
    for lev in range(1, depth + 1):
        for c in np.nonzero(d.level == lev)[0]:
            p = int(d.parent[c])
            if rank(c) == 0 or rank(p) == 0:
                continue
            yh[int(c)] = (yh[int(c)] + mul(_block_operand(tier, "transfer", transfer(c)),
                                           _coef_operand(tier, yh[p]))).astype(np.complex64)
    # leaves: the inadmissible blocks, then the backward transformation V_t y^_t,
    # in one accumulator per leaf
    y = np.zeros_like(U32)
    acc = {c: zero(size(c)) for c in range(nc) if d.nchild[c] == 0}
    for i in range(d.near_t.shape[0]):
        t, s = int(d.near_t[i]), int(d.near_s[i])
        G = _block(d.near, int(d.near_off[i]), size(t), size(s))
        acc[t] = (acc[t] + mul(_block_operand(tier, "near", G), Uop[s])).astype(np.complex64)
    for c in acc:
        if rank(c) > 0:
            acc[c] = (acc[c] + mul(_block_operand(tier, "basis", basis(c)),
                                 _coef_operand(tier, yh[c]))).astype(np.complex64)
        y[d.begin[c]:d.end[c]] = acc[c]
    return y


def h2_matvec_tier(d, x: np.ndarray, tier: str, op: str = "Z") -> np.ndarray:
    """The tier's product on x of shape (3 n_vox,) or (3 n_vox, nrhs), caller ordering.

    Returns complex64.  op "G" gives (G (x) I_3) x, op "Z" gives
    x + sigma k^2 V (G (x) I_3)(chi . x), all in float32."""
    if tier not in _MUL:
        raise ValueError(tier)
    n = int(d.n_vox)
    X = np.asarray(x).astype(np.complex64).reshape(n, -1)
    if op == "G":
        U = X
    else:
        chi = np.asarray(d.chi).astype(np.complex64)
        U = (chi[:, None] * X).astype(np.complex64)
    y_tree = _apply_tier(d, np.ascontiguousarray(U[d.perm]), tier)
    Y = np.empty_like(y_tree)
    Y[d.perm] = y_tree
    if op == "G":
        return Y.reshape(np.shape(x))
    alpha = np.float32(d.sigma * d.k * d.k * d.volume)
    return (X + alpha * Y).astype(np.complex64).reshape(np.shape(x))
