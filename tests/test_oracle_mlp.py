"""Pins of the FP64 surrogate reference and of the precision codec.

* backpropagation against central finite differences of the loss;
* the network reduces to its output bias when the hidden weights vanish, to
  the affine map W3 (W2 (W1 x + b1) + b2) + b3 when every unit is active, and
  to a constant when the first layer is inactive (ReLU);
* Adam: the first step from zero moments moves each parameter by lr sign(g);
* BF16 round-to-nearest-even on hand-built bit patterns (halfway cases tie
  to even) and against an FP64 nearest-value search; FP16 against known
  patterns;
* deviation codec round trip error bounded by half an ulp of the deviation.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_2510_14712_amd import inputs


def _batch(n=17, seed=5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (n, 2)), rng.normal(size=(n, 3))


def test_backprop_matches_finite_differences():
    params = inputs.mlp_params(7, scale=1.5)
    params[64 * 2:64 * 3] = np.random.default_rng(1).normal(size=64) * 0.3   # nonzero b1
    xn, tn = _batch()
    L, g = mlp.loss_grad(params, xn, tn)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [0, 128, 4546, 4545]])
    h = 1e-6
    for i in idx:
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd = (mlp.loss_grad(pp, xn, tn)[0] - mlp.loss_grad(pm, xn, tn)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(fd) + 2e-9


def test_forward_special_cases():
    xn, _ = _batch()
    # hidden weights zero: the output bias
    p = np.zeros(mlp.N_PARAMS)
    p[-3:] = [0.5, -1.0, 2.0]
    y, _ = mlp.forward(p, xn)
    np.testing.assert_array_equal(y, np.tile([0.5, -1.0, 2.0], (xn.shape[0], 1)))
    # every pre-activation positive: the affine map W3 (W2 (W1 x + b1) + b2) + b3
    rng = np.random.default_rng(11)
    W1 = rng.uniform(0.1, 1.0, (64, 2)); b1 = np.full(64, 3.0)
    W2 = rng.uniform(0.0, 0.1, (64, 64)); b2 = rng.uniform(0.1, 1.0, 64)
    W3 = rng.normal(size=(3, 64)); b3 = rng.normal(size=3)
    q = mlp.pack(W1, b1, W2, b2, W3, b3)
    y, (x, h1, h2) = mlp.forward(q, xn)
    assert (xn @ W1.T + b1).min() > 0 and h1.min() > 0 and h2.min() > 0
    np.testing.assert_allclose(y, (((xn @ W1.T + b1) @ W2.T + b2) @ W3.T + b3), rtol=1e-13, atol=1e-13)
    # every first-layer pre-activation negative: the layers above see zeros
    q = mlp.pack(W1, -b1, W2, b2, W3, b3)
    y, _ = mlp.forward(q, xn)
    np.testing.assert_allclose(y, np.tile(np.maximum(b2, 0) @ W3.T + b3, (xn.shape[0], 1)), rtol=1e-13)


def test_adam_first_step():
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)
    np.testing.assert_allclose(p1 - p, -1e-3 * np.sign(g), rtol=1e-4)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rne_patterns():
    one = np.float32(1.0)
    ulp = 2.0 ** -7  # bf16 spacing at 1
    cases = {
        1.0: 0x3F80,
        1.0 + ulp: 0x3F81,
        1.0 + ulp / 2: 0x3F80,          # halfway, tie to even (0x3F80)
        1.0 + 3 * ulp / 2: 0x3F82,      # halfway, tie to even (0x3F82)
        1.0 + ulp / 2 + 2.0 ** -20: 0x3F81,
        -2.0: 0xC000,
        0.0: 0x0000,
    }
    for val, bits in cases.items():
        assert int(mlp.bf16_bits(np.float32(val))) == bits, val
    assert int(mlp.bf16_bits(np.float32(np.inf))) == 0x7F80
    assert np.isnan(mlp.bf16_to_f32(mlp.bf16_bits(np.float32(np.nan))))
    del one


def test_bf16_nearest_by_search():
    rng = np.random.default_rng(9)
    x = (rng.normal(size=4000) * 10.0 ** rng.uniform(-6, 3, 4000)).astype(np.float32)
    got = mlp.bf16_to_f32(mlp.bf16_bits(x)).astype(np.float64)
    # candidates: truncation and the next bf16 value away from zero
    u = x.view(np.uint32)
    lo = ((u >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    hi = (((u >> 16) + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo, dhi = np.abs(xd - lo), np.abs(hi - xd)
    expect = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi,
                      np.where(((u >> 16) & 1) == 0, lo, hi)))
    np.testing.assert_array_equal(got, expect)


def test_f16_patterns():
    assert int(mlp.f16_bits(np.float32(1.0))) == 0x3C00
    assert int(mlp.f16_bits(np.float32(1.0 + 2.0 ** -11))) == 0x3C00   # tie to even
    assert int(mlp.f16_bits(np.float32(1.0 + 3 * 2.0 ** -11))) == 0x3C02
    assert int(mlp.f16_bits(np.float32(-0.5))) == 0xB800
    assert int(mlp.f16_bits(np.float32(65504.0))) == 0x7BFF


@pytest.mark.parametrize("kind,ulp_rel", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_deviation_round_trip(kind, ulp_rel):
    rng = np.random.default_rng(10)
    ref = rng.uniform(0.01, 3.0, 1000).astype(np.float32)
    f = (ref * (1 + rng.uniform(-0.2, 0.2, 1000))).astype(np.float32)
    back = mlp.decode_deviation(mlp.encode_deviation(f, ref, kind), ref, kind)
    d = np.abs(f.astype(np.float64) - ref.astype(np.float64))
    err = np.abs(back.astype(np.float64) - f.astype(np.float64))
    # half an ulp of d is at most 2^-8 d (bf16) or 2^-11 d (fp16); plus the FP32 add
    assert np.all(err <= d * ulp_rel * 1.0001 + np.abs(f) * 2.0 ** -23 + 1e-30)
