"""Pins of the precision-tier emulation (P9).

Most pins use a hand-built seven-cluster description: a root of rank 0, two
rank-1 clusters that form an admissible pair, four one-voxel rank-1 leaves, and
two more couplings from leaf 5 to leaves 3 and 4 (zero unless a case sets them;
the description is a product definition here, not a partition).  Every block is
1x1, so each output is a closed form of a few products (tree order = voxel
order, leaves 3..6 hold voxels 0..3, x^_c and y^_c are cluster coefficients):

  y_0 = G_33 u_0 + G_34 u_1 + V_3 T_3 S_12 (T_5 V_5 u_2 + T_6 V_6 u_3)
  y_2 = G_55 u_2 + G_56 u_3 + V_5 (S_53 x^_3 + S_54 x^_4 + T_5 S_21 (T_3 x^_3 + T_4 x^_4)),
  x^_3 = V_3 u_0,  x^_4 = V_4 u_1

With u = (b, 0, 0, 0) and the blocks 1 except the ones a case sets, the tier's
output is worked out by hand below.  The values are powers of two and short sums
of them, so every float32 operation the emulation performs is exact except the
roundings each case is about; the expected values are therefore exact.
"""
import numpy as np
import pytest

from h2gen.desc import H2Desc
from oracle import matvec as om
from oracle import precision as op

F32 = np.float32


def tiny_desc(**vals):
    """The seven-cluster description with 1x1 blocks, all 1 unless given.

    Names: G33 G34 G43 G44 G55 G56 G65 G66 (near), S12 S21 S53 S54 (couplings;
    S53 and S54 default to 0), V3..V6 (leaf bases), T3..T6 (transfers)."""
    near_pairs = [(3, 3), (3, 4), (4, 3), (4, 4), (5, 5), (5, 6), (6, 5), (6, 6)]
    near = np.array([vals.get(f"G{t}{s}", 1.0) for t, s in near_pairs], np.complex128)
    coupling = np.array([vals.get("S12", 1.0), vals.get("S21", 1.0), vals.get("S53", 0.0), vals.get("S54", 0.0)],
                        np.complex128)
    basis = np.array([vals.get(f"V{c}", 1.0) for c in (3, 4, 5, 6)], np.complex128)
    transfer = np.array([vals.get(f"T{c}", 1.0) for c in (3, 4, 5, 6)], np.complex128)
    i32 = lambda a: np.array(a, np.int32)
    i64 = lambda a: np.array(a, np.int64)
    return H2Desc(
        n_vox=4, ncomp=3, perm=i32([0, 1, 2, 3]),
        level=i32([0, 1, 1, 2, 2, 2, 2]), parent=i32([-1, 0, 0, 1, 1, 2, 2]),
        begin=i64([0, 0, 2, 0, 1, 2, 3]), end=i64([4, 2, 4, 1, 2, 3, 4]),
        first_child=i32([1, 3, 5, -1, -1, -1, -1]), nchild=i32([2, 2, 2, 0, 0, 0, 0]),
        rank=i32([0, 1, 1, 1, 1, 1, 1]),
        basis_off=i64([-1, -1, -1, 0, 1, 2, 3]), basis=basis,
        transfer_off=i64([-1, -1, -1, 0, 1, 2, 3]), transfer=transfer,
        far_t=i32([1, 2, 5, 5]), far_s=i32([2, 1, 3, 4]), far_off=i64([0, 1, 2, 3]), coupling=coupling,
        near_t=i32([t for t, _ in near_pairs]), near_s=i32([s for _, s in near_pairs]),
        near_off=i64(range(8)), near=near,
        chi=np.ones(4, np.complex128), k=2 * np.pi, volume=1e-3, sigma=1.0)


def run(tier, d, u0, comp=0, u1=0.0):
    x = np.zeros(12, np.complex128)
    x[comp] = u0
    x[3 + comp] = u1
    y = op.h2_matvec_tier(d, x, tier, "G")
    return y.reshape(4, 3)[:, comp]


Q = 1 + 2.0 ** -9 + 2.0 ** -20      # float32-exact; hi = 1, lo = bf16(2^-9 + 2^-20) = 2^-9
Q_BF = 1 + 2.0 ** -9                 # what the BF16 tier keeps of Q
P = 1 + 2.0 ** -30                   # float32 keeps 1
A = 1 + 2.0 ** -7                    # bf16-exact (lo = 0)
B = 1 + 2.0 ** -9 + 2.0 ** -16       # hi = 1, lo = 2^-9 (1 + 2^-7), both exact: kept whole
AB = 1 + 2.0 ** -7 + 2.0 ** -9 + 2.0 ** -15 + 2.0 ** -23   # A*B, exact in float32 (24 bits)
AB_SPLIT = 1 + 2.0 ** -7 + 2.0 ** -9 + 2.0 ** -15           # hi(AB) = A, lo(AB) = bf16(2^-9 + 2^-15 + 2^-23)
R = 1 + 2.0 ** -9                    # hi = 1, lo = 2^-9: R*R = 1 + 2^-8 + 2^-18, lo*lo = 2^-18


def test_closed_form_constants():
    # the bit-level facts the cases rest on, checked against torch's own bfloat16 conversion
    import torch
    bf = lambda v: float(torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).float())
    assert bf(Q) == 1.0 and bf(np.float32(Q) - 1.0) == 2.0 ** -9
    assert bf(B) == 1.0 and bf(np.float32(B) - 1.0) == np.float32(B) - 1.0
    assert bf(A) == A and float(F32(A) * F32(B)) == AB
    assert bf(F32(AB)) == A and bf(F32(AB) - F32(A)) == 2.0 ** -9 + 2.0 ** -15
    assert float(F32(P)) == 1.0 and float(F32(Q)) == Q


def test_bf16_round_matches_torch():
    import torch
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


# ---------------------------------------------------------------- closed forms
def test_fp64_closed_form_of_the_tiny_description():
    # the FP64 oracle on the same description, as the module docstring writes it
    d = tiny_desc(G33=2.0, G43=3.0, V3=5.0, T3=7.0, S21=11.0, T5=13.0, V5=17.0, T6=19.0, V6=23.0)
    x = np.zeros(12, np.complex128)
    x[0] = 1.0
    y = om.h2_matvec(d, x, "G").reshape(4, 3)[:, 0]
    assert np.array_equal(y, [2.0, 3.0, 5 * 7 * 11 * 13 * 17, 5 * 7 * 11 * 19 * 23])


# Each block of the path u_0 -> y_2 set to Q in turn: the tier keeps Q_BF of it.
PATH = ["V3", "T3", "S21", "T5", "V5"]


@pytest.mark.parametrize("name", PATH)
def test_bf16_block_rounding_on_far_path(name):
    y = run("bf16x3", tiny_desc(**{name: Q}), 1.0)
    assert y[2] == F32(Q_BF) and y[0] == 1.0


def test_bf16_near_block_and_vector_rounding():
    y = run("bf16x3", tiny_desc(G33=Q, G43=Q), 1.0)
    assert y[0] == F32(Q_BF) and y[1] == F32(Q_BF) and y[2] == 1.0
    y = run("bf16x3", tiny_desc(), Q)          # x itself
    assert y[0] == F32(Q_BF) and y[2] == F32(Q_BF)
    y = run("bf16x3", tiny_desc(), 1j * Q)     # imaginary parts are split alike
    assert y[0] == np.complex64(1j * Q_BF) and y[2] == np.complex64(1j * Q_BF)


@pytest.mark.parametrize("name", PATH + ["G33"])
def test_fp32_block_rounding(name):
    y = run("fp32", tiny_desc(**{name: P}), 1.0)
    assert y[2 if name != "G33" else 0] == 1.0
    y = run("fp32", tiny_desc(**{name: Q}), 1.0)   # Q is float32-exact: kept whole
    assert y[2 if name != "G33" else 0] == F32(Q)


def test_bf16_drops_lo_times_lo():
    # R*R in three terms: 1 + 2^-8 (the exact product has another 2^-18)
    y = run("bf16x3", tiny_desc(G33=R, V3=R), R)
    assert y[0] == F32(1 + 2.0 ** -8)
    assert y[2] == F32(1 + 2.0 ** -8)          # x^_3 = V3 u_0, then exact steps


# A on one block of the path, B at the input: the product A*B needs 24 bits, and the
# next step sees its hi + lo split (AB_SPLIT); on the last step (V5) nothing follows.
@pytest.mark.parametrize("name,expect", [("V3", AB_SPLIT), ("T3", AB_SPLIT), ("S21", AB_SPLIT),
                                         ("T5", AB_SPLIT), ("V5", AB)])
def test_bf16_coefficients_resplit_between_steps(name, expect):
    y = run("bf16x3", tiny_desc(**{name: A}), B)
    assert y[2] == F32(expect)


# Cancellation exposes what a rounding removed: Q on one block, a -1 term beside it,
# the difference 2^-9 (rounded Q) or 2^-9 + 2^-20 (Q kept whole) survives the re-split.
CANCEL = {"V3": dict(V3=Q), "T3": dict(T3=Q), "S53": dict(S53=Q, S54=1.0), "T5": dict(T5=Q, S53=-1.0)}


@pytest.mark.parametrize("name", list(CANCEL))
def test_bf16_rounding_survives_cancellation(name):
    u1 = 0.0 if name == "T5" else -1.0
    y = run("bf16x3", tiny_desc(**CANCEL[name]), 1.0, u1=u1)
    assert y[2] == F32(2.0 ** -9), y[2]


def test_fp32_keeps_coefficients_whole():
    for name in ("V3", "T3", "S21", "T5", "V5"):
        assert run("fp32", tiny_desc(**{name: A}), B)[2] == F32(AB)


def test_fp32_accumulates_in_float32():
    # leaf 3 sums G33 u_0 = 1, then G34 u_1 = 2^-24, then V3 y^_3 = 2^-24 (from u_2) in one
    # float32 accumulator: each 2^-24 is half an ulp of 1 and rounds away (ties to even).
    d = tiny_desc()
    x = np.zeros(12, np.complex128)
    x[0], x[3], x[6] = 1.0, 2.0 ** -24, 2.0 ** -24
    for tier in ("fp32", "bf16x3"):
        y = op.h2_matvec_tier(d, x, tier, "G").reshape(4, 3)[:, 0]
        assert y[0] == 1.0, tier
    assert om.h2_matvec(d, x, "G").reshape(4, 3)[0, 0] == 1 + 2.0 ** -23   # FP64 keeps both


def test_op_z_rounds_chi_and_scale():
    d = tiny_desc()
    d.chi = np.array([P, 1, 1, 1], np.complex128)
    d.sigma, d.k, d.volume = 1.0, 1.0, P          # sigma k^2 V = P in FP64, 1 in float32
    x = np.zeros(12, np.complex128)
    x[0] = 1.0
    y = op.h2_matvec_tier(d, x, "fp32", "Z").reshape(4, 3)[:, 0]
    # y_0 = x_0 + 1 * (G33 * 1 + 0) = 2, y_2 = 0 + 1 * 1 = 1
    assert y[0] == 2.0 and y[2] == 1.0


# ---------------------------------------------------------------- structure
def _integer_desc(name, seed):
    """A built description with every block entry replaced by a small complex integer."""
    from conftest import built
    import copy
    g, d = built(name)
    e = copy.copy(d)
    rng = np.random.default_rng(seed)
    vals = np.array([0, 1, -1, 1j, -1j], np.complex128)
    for arr in ("near", "coupling", "basis", "transfer"):
        a = getattr(d, arr)
        setattr(e, arr, rng.choice(vals, size=a.shape, p=[0.84, 0.04, 0.04, 0.04, 0.04]))
    return g, e


@pytest.mark.parametrize("name", ["rod", "cube12"])
@pytest.mark.parametrize("tier", ["fp32", "bf16x3"])
def test_tier_equals_fp64_when_everything_is_representable(name, tier):
    # small integers: every stored value is bf16-exact with lo = 0 and every partial sum
    # is an integer far below 2^24, so both tiers must return the FP64 oracle exactly.
    # This pins the structure (which blocks, which transposes, which sums) to the FP64
    # oracle, itself pinned to dense G.
    g, e = _integer_desc(name, 5)
    rng = np.random.default_rng(6)
    x = np.zeros(3 * g.n_vox, np.complex128)
    x[rng.choice(3 * g.n_vox, 6, replace=False)] = [1, -1, 1j, 2, -2j, 1 + 1j]
    y64 = om.h2_matvec(e, x, "G")
    yt = op.h2_matvec_tier(e, x, tier, "G")
    assert np.count_nonzero(y64) > g.n_vox          # the far and near paths both reach the output
    assert np.array_equal(yt.astype(np.complex128), y64)


def test_tier_errors_ordered():
    from conftest import built
    import h2gen
    g, d = built("cube12")
    x = h2gen.random_vector(3 * g.n_vox, 1)
    y = om.h2_matvec(d, x)
    e32 = np.linalg.norm(op.h2_matvec_tier(d, x, "fp32") - y) / np.linalg.norm(y)
    e16 = np.linalg.norm(op.h2_matvec_tier(d, x, "bf16x3") - y) / np.linalg.norm(y)
    assert 1e-9 < e32 < 1e-6 and e32 < e16 < 1e-4


# ---------------------------------------------------------------- planted mistakes
def _fails(test, *args):
    try:
        test(*args)
    except AssertionError:
        return True
    return False


def test_planted_missing_resplit_is_caught(monkeypatch):
    keep = lambda tier, c: op._OPERAND[tier](c) if tier == "fp32" else _whole(c)
    monkeypatch.setattr(op, "_coef_operand", keep)
    for name in ("V3", "T3", "S21", "T5"):
        assert _fails(test_bf16_coefficients_resplit_between_steps, name, AB_SPLIT), name


def _whole(v):
    """A BF16 operand that (wrongly) carries its float32 value whole in hi."""
    o = op._SplitOperand(np.zeros(np.shape(v), np.complex64))
    o.hi = np.asarray(v).astype(np.complex64)
    return o


@pytest.mark.parametrize("which", ["near", "coupling", "basis", "transfer"])
def test_planted_unrounded_block_array_is_caught(monkeypatch, which):
    real = op._block_operand

    def wrong(tier, w, B):
        return _whole(B) if (tier == "bf16x3" and w == which) else real(tier, w, B)

    monkeypatch.setattr(op, "_block_operand", wrong)
    if which == "near":
        assert _fails(test_bf16_near_block_and_vector_rounding)
    else:
        names = {"coupling": ["S53"], "basis": [], "transfer": ["T3", "T5"]}[which]
        for name in names:
            assert _fails(test_bf16_rounding_survives_cancellation, name), name
    if which == "basis":
        assert _fails(test_bf16_block_rounding_on_far_path, "V5")


def test_planted_unsplit_vector_is_caught(monkeypatch):
    monkeypatch.setattr(op, "_vector_operand", lambda tier, u: _whole(u) if tier == "bf16x3" else op._Fp32Operand(u))
    assert _fails(test_bf16_near_block_and_vector_rounding)


def test_planted_lo_times_lo_is_caught(monkeypatch):
    def four_terms(a, b):
        return (a.hi @ b.hi + a.hi @ b.lo + a.lo @ b.hi + a.lo @ b.lo).astype(np.complex64)
    monkeypatch.setitem(op._MUL, "bf16x3", four_terms)
    assert _fails(test_bf16_drops_lo_times_lo)


def test_planted_wide_accumulator_is_caught(monkeypatch):
    # the blocks rounded to the tier but every sum carried in complex128 until the end
    import copy

    def wide(d, U32, tier):
        e = copy.copy(d)
        for arr in ("near", "coupling", "basis", "transfer"):
            setattr(e, arr, np.asarray(getattr(d, arr)).astype(np.complex64).astype(np.complex128))
        return om.h2_apply_tree(e, U32.astype(np.complex128)).astype(np.complex64)

    monkeypatch.setattr(op, "_apply_tier", wide)
    assert _fails(test_fp32_accumulates_in_float32)


@pytest.mark.parametrize("which", ["coupling", "basis", "transfer", "near"])
def test_planted_conjugate_is_caught(monkeypatch, which):
    # the construction uses conjugate transposes, the product plain ones: a conjugate
    # slipped into the product must break the structure pin
    real = op._block_operand
    monkeypatch.setattr(op, "_block_operand", lambda tier, w, B: real(tier, w, B.conj() if w == which else B))
    geom = "rod" if which == "transfer" else "cube12"    # cube12 has no transfers
    assert _fails(test_tier_equals_fp64_when_everything_is_representable, geom, "bf16x3")
