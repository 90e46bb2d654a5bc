"""Pins for the wavelet oracle (LeGall 5/3 integer lifting, two levels on
8x8 blocks, Sec. 6.8-6.9): hand-computed lifting results, exact
invertibility, the value ranges the report prints (Sec. 6.9.4), constant
blocks, and the fragment round trip with the pinned AES-CTR."""
import numpy as np

import oracle
import synth
from oracle import dwt


def test_lifting_hand_examples():
    # d(i) = x(2i+1) - floor((x(2i) + x(2i+2)) / 2), x(8) = x(6);
    # s(i) = x(2i) + floor((d(i-1) + d(i) + 2) / 4), d(-1) = d(0)
    assert dwt.lift_forward(np.arange(8)).tolist() == [0, 2, 4, 6, 0, 0, 0, 1]
    assert dwt.lift_forward(np.full(8, 5)).tolist() == [5, 5, 5, 5, 0, 0, 0, 0]
    # alternating signal: d = 0 - 10 = -10 everywhere, s = 10 + floor(-18 / 4) = 5
    assert dwt.lift_forward(np.array([10, 0] * 4)).tolist() == [5, 5, 5, 5, -10, -10, -10, -10]
    # 4-point (second level): x = [1, 4, 9, 16]: d0 = 4 - 5 = -1, d1 = 16 - 9 = 7 (x(4) = x(2));
    # s0 = 1 + floor((-1 - 1 + 2) / 4) = 1, s1 = 9 + floor((-1 + 7 + 2) / 4) = 11
    assert dwt.lift_forward(np.array([1, 4, 9, 16])).tolist() == [1, 11, -1, 7]


def test_lifting_is_exactly_invertible():
    rng = np.random.default_rng(0)
    for n in (4, 8):
        x = rng.integers(-600, 600, size=(5000, n))
        assert np.array_equal(dwt.lift_inverse(dwt.lift_forward(x)), x)
    b = rng.integers(0, 256, size=(5000, 64))
    assert np.array_equal(dwt.idwt_blocks(dwt.dwt_blocks(b)), b)


def test_constant_block_has_only_the_low_low_values():
    # the low-pass filter has unit gain: a constant block leaves x - 128 in
    # each of the four second-level low-low coefficients and zero elsewhere
    for v in (0, 37, 128, 255):
        c = dwt.dwt_blocks(np.full((1, 64), v))[0]
        assert np.all(c[:2, :2] == v - 128)
        c[:2, :2] = 0
        assert not c.any()


def _linear_bound():
    """128 * sum_p |w_p| per coefficient: the weights of the two-level
    transform, measured on impulses of height 2^30 (the floors then move a
    weight by less than 2^-29)."""
    scale = float(1 << 30)
    w = np.zeros((64, 8, 8))
    for p in range(64):
        e = np.zeros((1, 8, 8), np.int64)
        e[0, p // 8, p % 8] = 1 << 30
        c = dwt.level_forward(e)
        c[:, :4, :4] = dwt.level_forward(c[:, :4, :4])
        w[p] = c[0] / scale
    return 128 * np.abs(w).sum(0)


def test_value_ranges_printed_in_the_report():
    # Sec. 6.9.4: first level LH within +-384, HH within +-511; second level
    # (4x4 low-low quarter) extremes 338 (low-low), 468, 648
    b = _linear_bound()
    assert abs(b[4, 0] - 384) < 1 and abs(b[0, 4] - 384) < 1
    assert abs(b[4, 4] - 511) <= 1.5
    assert abs(b[0, 0] - 338) < 1
    assert abs(b[0, 2] - 468) < 1 and abs(b[2, 0] - 468) < 1
    assert abs(b[2, 2] - 648) < 1 and abs(b[3, 3] - 648) < 1
    # extremal 0/255 inputs reach the bounds (up to the one-sided byte range and floors)
    # and never exceed them
    rng = np.random.default_rng(1)
    x = rng.integers(0, 2, size=(20000, 64)) * 255
    c = np.abs(dwt.dwt_blocks(x))
    assert np.all(c <= b + 1)


def test_fragments_round_trip_and_cipher():
    x = synth.image(24, 40, 3, 2, 0).numpy()
    key, c0 = synth.aes_key(2), synth.ctr0(2, 0)
    f = dwt.frag(x, key, c0)
    nb = 3 * 3 * 5
    assert f["public"].size == 60 * nb and f["private"].size == 4 * nb
    assert np.array_equal(f["cipher"], oracle.ctr_xor(key, c0, f["private"].view(np.uint8)))
    y = dwt.defrag(x.shape, f["public"], key=key, ctr0=c0, cipher=f["cipher"])
    assert np.array_equal(y, x)
    # the private values are the second-level low-low corners, block by block
    c = dwt.dwt_blocks(oracle.blocks_of(x))
    priv = oracle.tile_unpack(f["private"], nb, 4)
    assert np.array_equal(priv[:, 0], c[:, 0, 0]) and np.array_equal(priv[:, 3], c[:, 1, 1])
