"""Emulation of the lower-precision storage tiers (test infrastructure).

* FP32 tier: every stored block entry rounded to complex64, vectors carried in
  complex64, products accumulated in float32.
* BF16 hi+lo tier: each real part v is split into hi = bf16(v) and
  lo = bf16(v - hi) with round-to-nearest-even; a product a*b is formed from
  the three terms hi_a hi_b + hi_a lo_b + lo_a hi_b (lo_a lo_b dropped), with
  float32 accumulation.

bf16 rounding is written out on the float32 bit pattern: add 0x7fff plus the
lowest kept bit, then clear the low 16 bits.
"""

from __future__ import annotations

import copy

import numpy as np

from . import matvec as om


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = ~np.isfinite(f)
    out = np.where(nan, f, out)
    return out


def split_bf16(z: np.ndarray):
    """(hi, lo) complex64 arrays with bf16-representable parts, hi + lo ~= z."""
    re = np.asarray(z.real, np.float32)
    im = np.asarray(z.imag, np.float32)
    hr, hm = bf16_round(re), bf16_round(im)
    lr, lm = bf16_round(re - hr), bf16_round(im - hm)
    return (hr + 1j * hm).astype(np.complex64), (lr + 1j * lm).astype(np.complex64)


def round_desc(d, tier: str):
    """Copy of an H2Desc whose block arrays hold the values the tier stores.

    For the BF16 tier the stored value is hi + lo (the three-term product keeps
    everything but lo*lo, which is below float32 rounding of the sum).
    """
    e = copy.copy(d)
    for name in ("near", "coupling", "basis", "transfer"):
        a = np.asarray(getattr(d, name))
        if tier == "fp32":
            v = a.astype(np.complex64)
        elif tier == "bf16x3":
            hi, lo = split_bf16(a)
            v = (hi.astype(np.complex128) + lo.astype(np.complex128)).astype(np.complex64)
        else:
            raise ValueError(tier)
        setattr(e, name, v)
    return e


def h2_matvec_tier(d, x: np.ndarray, tier: str, op: str = "Z") -> np.ndarray:
    """Product with the tier's stored blocks, vectors in complex64 (float32 accumulation)."""
    e = round_desc(d, tier)
    e.chi = np.asarray(d.chi).astype(np.complex64)
    x32 = np.asarray(x).astype(np.complex64)
    if tier == "bf16x3":
        hi, lo = split_bf16(x32)
        x32 = (hi.astype(np.complex128) + lo.astype(np.complex128)).astype(np.complex64)
    n = int(d.n_vox)
    X = x32.reshape(n, -1)
    U = X if op == "G" else e.chi[:, None] * X
    y_tree = om.h2_apply_tree(e, U[d.perm])
    Y = np.empty_like(y_tree)
    Y[d.perm] = y_tree
    if op == "G":
        return Y.reshape(x.shape)
    alpha = np.float32(d.sigma * d.k * d.k * d.volume)
    return (X + alpha * Y).reshape(x.shape)
