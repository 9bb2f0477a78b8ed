"""Pins of the precision-tier emulation (P9)."""
import numpy as np
import torch

from oracle import precision as op


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([1.0, 1.00390625, 1.01171875, -2.5, 0.0, 65504.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(op.bf16_round(x), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert op.bf16_round(np.array([1.00390625], np.float32))[0] == 1.0
    assert op.bf16_round(np.array([1.01171875], np.float32))[0] == 1.015625


def test_split_hi_lo_accuracy():
    rng = np.random.default_rng(1)
    z = (rng.standard_normal(5000) + 1j * rng.standard_normal(5000)).astype(np.complex128)
    hi, lo = op.split_bf16(z)
    rel = np.abs((hi.astype(np.complex128) + lo) - z) / np.abs(z)
    assert rel.max() < 2.0 ** -15          # two bf16 terms carry ~16 bits
    assert np.all(op.bf16_round(hi.real) == hi.real) and np.all(op.bf16_round(lo.imag) == lo.imag)


def test_tier_errors_ordered():
    from conftest import built
    import h2gen
    from oracle import matvec as om
    g, d = built("cube12")
    x = h2gen.random_vector(3 * g.n_vox, 1)
    y = om.h2_matvec(d, x)
    e32 = np.linalg.norm(op.h2_matvec_tier(d, x, "fp32") - y) / np.linalg.norm(y)
    e16 = np.linalg.norm(op.h2_matvec_tier(d, x, "bf16x3") - y) / np.linalg.norm(y)
    assert 1e-9 < e32 < 1e-6 and e32 < e16 < 1e-4
