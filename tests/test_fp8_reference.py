"""Pins of the test-side fp8 operand-rounding model (tests/fp8_reference.py):
the E4M3 grid and its ties, the MX block exponent, the polyphase form of the
upsampling convs against the oracle's upsample-then-conv, and the exactness
of MX quantisation on values that are already representable."""
import numpy as np

import synth
from oracle import tokenizer as O
from tests import fp8_reference as F8


def _e4m3_grid():
    """Every positive finite OCP E4M3 value from its bit fields (bias 7;
    exponent field 0 = subnormal; S.1111.111 is NaN, so 448 is the largest)."""
    vals = []
    for ef in range(16):
        for m in range(8):
            if ef == 15 and m == 7:
                continue
            vals.append(m / 8 * 2.0 ** -6 if ef == 0 else (1 + m / 8) * 2.0 ** (ef - 7))
    return np.array(sorted(vals))


def test_e4m3_grid_is_fixed_and_ties_go_to_even():
    g = _e4m3_grid()
    assert g[0] == 0.0 and g[-1] == 448.0 and g[1] == 2.0 ** -9 and len(g) == 127
    np.testing.assert_array_equal(F8.e4m3(g), g)
    np.testing.assert_array_equal(F8.e4m3(-g), -g)
    mids = (g[:-1] + g[1:]) / 2
    got = F8.e4m3(mids)
    # a midpoint rounds to the neighbour whose mantissa field is even
    lo_idx = np.arange(len(g) - 1)
    lo_even = np.array([round((v / (2.0 ** max(np.frexp(v)[1] - 1, -6) / 8)) if v > 0 else 0) % 2 == 0
                        for v in g[:-1]])
    np.testing.assert_array_equal(got, np.where(lo_even, g[lo_idx], g[lo_idx + 1]))
    # anything else goes to the nearest grid value
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 448, 20000)
    nearest = g[np.abs(x[:, None] - g[None, :]).argmin(axis=1)]
    np.testing.assert_array_equal(F8.e4m3(x), nearest)
    assert F8.e4m3(np.array([1.0625]))[0] == 1.0 and F8.e4m3(np.array([1.1875]))[0] == 1.25
    assert F8.e4m3(np.array([2.0 ** -10]))[0] == 0.0          # half the smallest subnormal: ties to 0


def test_block_exponent():
    am = np.array([448.0, 448.01, 224.0, 224.1, 1.0, 0.0, 3.0e-30, 896.0], np.float32)
    e = F8.block_exp(am)
    np.testing.assert_array_equal(e[:6], [0, 1, -1, 0, -8, 0])
    assert e[7] == 1
    # in general the smallest e with max * 2^-e <= 448, up to the rounding of max * fp32(1/448)
    rng = np.random.default_rng(1)
    a = (10.0 ** rng.uniform(-6, 6, 5000)).astype(np.float32)
    e = F8.block_exp(a)
    assert (a.astype(np.float64) * 2.0 ** -e.astype(np.float64) <= 448.0 * (1 + 2 ** -22)).all()
    assert (a.astype(np.float64) * 2.0 ** -(e.astype(np.float64) - 1) > 448.0 * (1 - 2 ** -22)).all()


def test_polyphase_upconv_equals_upsample_then_conv():
    x = synth.randn(2, (2, 3, 5, 6, 8)).astype(np.float64)
    w = synth.randn(3, (4, 8, 3, 3, 3)).astype(np.float64)
    b = synth.randn(4, (4,)).astype(np.float64)
    ref = O.conv3d(O.upsample(x), w, b)
    got = F8.upconv_poly(x, F8.fold_up(w, np.float64), b)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_mx_quantisation_is_exact_on_representable_values():
    rng = np.random.default_rng(5)
    g = _e4m3_grid()
    # per 32-channel block: grid values times one power of two, block maximum 448 * 2^k
    k = rng.integers(-20, 20, (7, 2))
    v = g[rng.integers(0, len(g), (7, 64))] * np.where(rng.uniform(size=(7, 64)) < 0.5, -1, 1)
    v[:, 0], v[:, 32] = 448.0, -448.0
    v = v * np.repeat(2.0 ** k, 32, axis=1)
    np.testing.assert_array_equal(F8.quantize_mx(v.astype(np.float32)), v)
    # and otherwise within half a quantum of the block's grid
    u = rng.standard_normal((50, 64)).astype(np.float32)
    q = F8.quantize_mx(u)
    e = F8.block_exp(np.abs(u.reshape(50, 2, 32)).max(-1))
    rel = np.abs(q - u).reshape(50, 2, 32) / 2.0 ** e[..., None]
    assert rel.max() <= 2.0 ** 5 / 2  # at most half the top binade's quantum (32) in scaled units


def test_weight_rounding_uses_per_channel_scales():
    w = synth.randn(6, (5, 7, 3, 3, 3)).astype(np.float32)
    q = F8.quant_s1(w)
    for c in range(5):
        s = np.float32(np.abs(w[c]).max() / np.float32(448.0))
        assert np.abs(q[c]).max() <= 448 * float(s) * (1 + 1e-6)
        grid = np.unique(np.abs(q[c] / float(s)))
        np.testing.assert_array_equal(F8.e4m3(grid), grid)


def test_accuracy_band_detects_a_rounding_mistake():
    """The fp8 GPU test's accuracy band (0.1 dB) against planted mistakes in
    the model on the CPU: truncating e4m3 instead of rounding to nearest even
    moves PSNR against the oracle by far more than the band, while evaluations
    that differ only in summation rounding stay inside it."""
    from tests import gpu_common as G
    ref = G.oracle_roundtrip((0,), 9, 64, 64, True)
    p = G.weights(True)
    base = O.psnr(F8.decode_fp8(ref["codes"], p), ref["xhat"])
    pert = O.psnr(F8.decode_fp8(ref["codes"], p, noise=(np.random.default_rng(3), 3e-5)), ref["xhat"])
    assert abs(pert - base) <= 0.1

    def truncating(x):
        x = np.asarray(x, np.float64)
        a = np.abs(x)
        _, ex = np.frexp(np.where(a > 0, a, 1.0))
        q = np.ldexp(1.0, np.maximum(ex - 1, -6) - 3)
        return np.where(a > 0, np.copysign(np.minimum(np.floor(a / q) * q, 448.0), x), 0.0)

    orig = F8.e4m3
    try:
        F8.e4m3 = truncating
        planted = O.psnr(F8.decode_fp8(ref["codes"], p), ref["xhat"])
    finally:
        F8.e4m3 = orig
    assert abs(planted - base) > 1.0, (planted, base)
