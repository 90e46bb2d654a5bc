"""Pins of the security-statistics oracle (oracle/stats.py): closed forms of
Eqs. (3)-(4), the report's printed values for random-looking data (Table 14),
scipy's entropy and Pearson routines, and hand cases."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import stats as st


def _blocks_image(blocks):
    """(8, 8) blocks side by side as one gray image."""
    return np.concatenate([np.asarray(b, np.uint8) for b in blocks], axis=1)[None]


def test_block_entropy_closed_forms():
    distinct = np.arange(64).reshape(8, 8)                   # Eq. (4): log2(64) = 6
    const = np.full((8, 8), 7)
    halves = np.indices((8, 8)).sum(0) % 2 * 200              # two values, 32 each: 1 bit
    quarters = (np.arange(64) % 4).reshape(8, 8) * 60         # four values, 16 each: 2 bits
    e = st.block_entropy(_blocks_image([distinct, const, halves, quarters]))
    assert np.allclose(e, [6.0, 0.0, 1.0, 2.0], atol=1e-15)


def test_expected_block_entropy_matches_the_report():
    # Table 14 / Sec. 6.10.3: the protected data's mean block entropy is 5.7656
    # (image) and 5.766 (text); for independent uniform bytes the expectation
    # has a closed form
    e = st.expected_block_entropy_uniform()
    assert abs(e - 5.7656) < 5e-4 and abs(e - 5.766) < 5e-4
    # and keystream bytes (AES-CTR of zeros) reach it within the sampling error
    ks = oracle.ctr_xor(bytes(range(16)), bytes(16), np.zeros(64 * 16384, np.uint8))
    be = st.block_entropy(ks.reshape(1, 8 * 128, 8 * 128))
    assert abs(be.mean() - e) < 5 * be.std() / math.sqrt(be.size)


def test_entropy_matches_scipy():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 50, 256)
    c[::7] = 0
    assert abs(st.entropy_bits(c) - scipy.stats.entropy(c, base=2)) < 1e-12


def test_chi2_uniformity():
    assert st.chi2_uniform(np.full(256, 1000)) == 0.0
    c = np.full(256, 100)
    c[0] += 50
    c[1] -= 50
    assert abs(st.chi2_uniform(c) - 2 * 2500 / 100) < 1e-12
    # uniform random bytes: chi2 ~ 255 +- sqrt(2 * 255) (Table 14 prints a mean of 256.08)
    ks = oracle.ctr_xor(bytes(16), bytes(16), np.zeros(1 << 20, np.uint8))
    assert abs(st.chi2_uniform(st.histogram(ks)) - 255) < 6 * math.sqrt(2 * 255)


def test_adjacent_correlation_against_scipy_and_hand_cases():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, (2, 40, 48)).astype(np.uint8)
    x = (x // 2 + np.roll(x, 1, axis=2) // 2).astype(np.uint8)     # some horizontal correlation
    for d in st.DIRS:
        u = np.concatenate([st.adjacent_pairs(x[c], d)[0].ravel() for c in range(2)])
        v = np.concatenate([st.adjacent_pairs(x[c], d)[1].ravel() for c in range(2)])
        assert abs(st.adjacent_correlation(x, d) - scipy.stats.pearsonr(u, v)[0]) < 1e-12
        assert st.pair_moments(x, d)[0] == u.size
    ramp = np.tile(np.arange(64, dtype=np.uint8), (16, 1))[None]    # x(r, c) = c
    assert abs(st.adjacent_correlation(ramp, "h") - 1.0) < 1e-12
    assert abs(st.adjacent_correlation(ramp, "v") - 1.0) < 1e-12     # pairs (c, c)
    assert st.adjacent_correlation(np.full((1, 8, 8), 3, np.uint8), "h") == 0.0   # zero variance guarded
    assert abs(st.adjacent_correlation(ramp, "d") - 1.0) < 1e-12
    # pairs never cross planes: two constant planes of different value
    two = np.stack([np.zeros((8, 8), np.uint8), np.full((8, 8), 9, np.uint8)])
    assert st.pair_moments(two, "v") == (112, 504, 504, 4536, 4536, 4536)   # no (0, 9) pair


def test_corr2_dif_psnr():
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, (1, 32, 32)).astype(np.uint8)
    y = (255 - x).astype(np.uint8)
    assert abs(st.corr2(x, x) - 1) < 1e-12 and abs(st.corr2(x, y) + 1) < 1e-12
    assert abs(st.corr2(x, rng.integers(0, 256, x.shape)) - np.corrcoef(x.ravel(), rng.integers(0, 256, x.size))[0, 1]) < 1
    assert st.bit_difference_percent(x, x) == 0.0 and st.bit_difference_percent(x, y) == 100.0
    assert st.bit_difference_percent(np.zeros(8, np.uint8), np.full(8, 0x0F, np.uint8)) == 50.0
    z = np.minimum(x.astype(int) + 1, 255)
    z[x == 255] = 254                                                 # every sample off by exactly 1
    assert abs(st.psnr(x, z) - 10 * math.log10(255 ** 2)) < 1e-12
    assert st.psnr(x, x) == float("inf")


def test_nmi_limits():
    rng = np.random.default_rng(11)
    x = rng.integers(0, 256, 1 << 18).astype(np.uint8)
    hx, hy, hxy, mi, n = st.nmi(x, x)
    assert abs(n - 1) < 1e-12 and abs(hxy - hx) < 1e-12
    perm = rng.permutation(256).astype(np.uint8)                      # a bijection keeps all information
    assert abs(st.nmi(x, perm[x])[4] - 1) < 1e-12
    y = rng.integers(0, 256, x.size).astype(np.uint8)                 # independent: only the plug-in bias
    bias = (255 * 255) / (2 * x.size * math.log(2))                   # E[I] of the plug-in estimate, bits
    assert st.nmi(x, y)[3] < 2 * bias and st.nmi(x, y)[4] < 2 * bias / 8
