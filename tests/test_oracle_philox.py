"""Pins of the oracle's Philox generator (the collision RNG contract)."""
import numpy as np
import pytest

from oracle.philox import PHILOX4x32, PHILOX4x64, philox4x32, philox_scalar, u32, u52


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((5, 7), (3, 0, 0, 0)),
                                     ((2 ** 64 - 1, 12345), (2 ** 63 + 11, 99, 2 ** 40, 1)),
                                     ((0xDEADBEEF, 0xFEEDFACE), (1, 2, 3, 4))])
def test_generic_philox_4x64_matches_numpy(key, ctr):
    # numpy.random.Philox is the 4x64-10 instance; it increments the counter
    # (with carry) before producing its first block.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = [int(v) for v in g.random_raw(8)]
    c = list(ctr)
    blocks = []
    for _ in range(2):
        c[0] = (c[0] + 1) % 2 ** 64
        if c[0] == 0:
            c[1] = (c[1] + 1) % 2 ** 64
        blocks += list(philox_scalar(c, key, PHILOX4x64))
    assert raw == blocks


def test_vectorised_4x32_matches_generic_scalar():
    g = np.random.Generator(np.random.PCG64(3))
    words = g.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    out = philox4x32(words[:, 0], words[:, 1], words[:, 2], words[:, 3], words[:, 4], words[:, 5])
    for i in range(200):
        ref = philox_scalar(words[i, :4], words[i, 4:], PHILOX4x32)
        assert tuple(int(o[i]) for o in out) == ref


def test_rounds_change_output():
    a = philox_scalar((1, 2, 3, 4), (5, 6), PHILOX4x32, rounds=10)
    b = philox_scalar((1, 2, 3, 4), (5, 6), PHILOX4x32, rounds=7)
    assert a != b


def test_4x32_uniformity_chi2_and_bit_balance():
    n = 1 << 16
    ctr = np.arange(n, dtype=np.uint64)
    r = philox4x32(ctr, 7, 0, 0, 12345, 0)
    u = np.concatenate([u32(w) for w in r])
    hist, _ = np.histogram(u, bins=256, range=(0.0, 1.0))
    expected = u.size / 256
    chi2 = float(np.sum((hist - expected) ** 2 / expected))
    # 255 degrees of freedom: mean 255, sd ~22.6; 6 sd either side.
    assert 120 < chi2 < 390
    words = np.concatenate(r).astype(np.uint64)
    for b in range(32):
        frac = float(np.mean((words >> np.uint64(b)) & np.uint64(1)))
        assert abs(frac - 0.5) < 6 * 0.5 / np.sqrt(words.size)


def test_4x32_avalanche():
    # Flipping one key bit changes about half of the 128 output bits.
    g = np.random.Generator(np.random.PCG64(9))
    flips = []
    for _ in range(200):
        c = [int(v) for v in g.integers(0, 2 ** 32, size=4)]
        k = [int(v) for v in g.integers(0, 2 ** 32, size=2)]
        a = philox_scalar(c, k, PHILOX4x32)
        bit = int(g.integers(0, 32))
        k2 = [k[0] ^ (1 << bit), k[1]]
        b = philox_scalar(c, k2, PHILOX4x32)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
    assert 60 < np.mean(flips) < 68


def test_uniform_maps_are_open_and_exact():
    assert u32(0) == 0.5 * 2.0 ** -32
    assert u32(2 ** 32 - 1) == 1.0 - 0.5 * 2.0 ** -32
    assert 0.0 < u52(0, 0) < 1.0
    top = u52(2 ** 32 - 1, 2 ** 32 - 1)
    assert top < 1.0 and top == 1.0 - 0.5 * 2.0 ** -52
