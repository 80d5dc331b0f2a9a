"""Checks of the seeded input generator (channel model, not the decoder)."""
import math

import numpy as np

from paper_1608_00066_amd import datagen


def test_noise_variance_formula():
    # rate 1/2 at 0 dB: Eb = 2, N0 = 2, sigma^2 = N0/2 = 1
    assert datagen.noise_variance(2, 0.0) == 1.0
    assert math.isclose(datagen.noise_variance(3, 10.0), 3 / 20)


def test_soft_quantizer_rounding_clip_and_sign():
    s2 = 2.0  # q = rint(8 y)
    y = np.array([0.3125, 0.1875, -0.3125, 100.0, -100.0, 0.0, 1e-9, -1e-9])
    q = datagen.quantize_soft(y, s2)
    # 8*0.3125 = 2.5 -> 2 (half to even), 8*0.1875 = 1.5 -> 2, clip at +-127
    assert q.tolist() == [2, 2, -2, 127, -127, 0, 0, 0]
    assert q.dtype == np.int8


def test_hard_quantizer():
    assert datagen.quantize_hard(np.array([0.5, -0.5, 0.0])).tolist() == [0, 1, 0]


def test_noiseless_channel_is_bpsk_full_scale():
    cb = np.array([[0, 1], [1, 1]], dtype=np.uint8)
    soft = datagen.channel(cb, None, np.random.default_rng(0), datagen.SOFT_I8)
    assert soft.view(np.int8).tolist() == [127, -127, -127, -127]
    hard = datagen.channel(cb, None, np.random.default_rng(0), datagen.HARD_U8)
    assert hard.tolist() == [0, 1, 1, 1]


def test_streams_are_seeded_and_sized():
    a = datagen.make_stream(7, (0o171, 0o133), 1000, 3.0, seed=5)
    b = datagen.make_stream(7, (0o171, 0o133), 1000, 3.0, seed=5)
    c = datagen.make_stream(7, (0o171, 0o133), 1000, 3.0, seed=6)
    assert np.array_equal(a["syms"], b["syms"]) and np.array_equal(a["info"], b["info"])
    assert not np.array_equal(a["syms"], c["syms"])
    assert a["T"] == 1006 and a["syms"].size == 1006 * 2
    u = datagen.make_stream(7, (0o171, 0o133), 1000, 3.0, seed=5, terminated=False)
    assert u["T"] == 1000


def test_channel_statistics():
    """Mean of y for bit 0 is +1 and its variance sigma^2 (checked on the
    quantized values through the 16/sigma^2 scale, away from the clip)."""
    R, ebn0 = 2, 2.0
    s2 = datagen.noise_variance(R, ebn0)
    cb = np.zeros((200000, R), dtype=np.uint8)
    q = datagen.channel(cb, ebn0, np.random.default_rng(1)).view(np.int8).astype(np.float64)
    y = q * s2 / 16.0
    assert abs(y.mean() - 1.0) < 0.02
    assert abs(y.var() - s2) / s2 < 0.05
