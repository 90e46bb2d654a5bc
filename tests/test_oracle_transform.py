"""Pins for the oracle's transform, zigzag, value ranges and integer quantiser.

Each test checks the oracle against something it does not compute itself:
scipy's DCT, closed forms of the orthonormal DCT-II, the report's own values
(Sec. 6.3.1 default selection, Sec. 6.4.3 DC bound), mpmath and brute force.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
from conftest import golden


def test_basis_orthonormal():
    B = oracle.basis()
    assert np.abs(B @ B.T - np.eye(64)).max() < 1e-14


def test_basis_dc_row_is_one_eighth():
    B = oracle.basis()
    assert np.abs(B[0] - 0.125).max() < 1e-16


def test_dct_matches_scipy_ortho():
    rng = np.random.default_rng(1)
    pix = rng.integers(0, 256, size=(2, 24, 40), dtype=np.uint8)
    C = oracle.dct_blocks(pix)
    blocks = oracle.blocks_of(pix).reshape(-1, 8, 8).astype(np.float64)
    ref = scipy.fft.dctn(blocks, type=2, norm="ortho", axes=(1, 2)).reshape(-1, 64)
    assert np.abs(C - ref).max() < 1e-11


def test_dct_closed_forms():
    # constant block -> only DC = 8 * value
    pix = np.full((1, 8, 8), 37, np.uint8)
    C = oracle.dct_blocks(pix)[0]
    assert abs(C[0] - 8 * 37) < 1e-12 and np.abs(C[1:]).max() < 1e-12
    # DC equals block sum / 8 on random data
    rng = np.random.default_rng(2)
    pix = rng.integers(0, 256, size=(1, 16, 16), dtype=np.uint8)
    C = oracle.dct_blocks(pix)
    S = oracle.blocks_of(pix).astype(np.int64).sum(1)
    assert np.abs(C[:, 0] - S / 8.0).max() < 1e-12


def test_basis_image_is_one_hot():
    B = oracle.basis()
    for n in (0, 1, 9, 27, 63):
        y = oracle.idct_blocks(np.eye(64)[n][None])[0]
        assert np.abs(y - B[n]).max() < 1e-15
    # scaled basis image transforms back to a one-hot vector
    rng = np.random.default_rng(3)
    n = 10
    coef = np.zeros((1, 64))
    coef[0, n] = 100.0
    y = oracle.idct_blocks(coef)[0]
    # undo through a direct (non-oracle) projection: sum_p y_p B[m, p]
    proj = B @ y
    assert np.abs(proj - coef[0]).max() < 1e-12
    del rng


def test_parseval_and_inverse():
    rng = np.random.default_rng(4)
    pix = rng.integers(0, 256, size=(1, 32, 32), dtype=np.uint8)
    C = oracle.dct_blocks(pix)
    X = oracle.blocks_of(pix).astype(np.float64)
    assert np.abs((C ** 2).sum(1) - (X ** 2).sum(1)).max() < 1e-7
    assert np.abs(oracle.idct_blocks(C) - X).max() < 1e-11


def test_zigzag_default_private_set_from_report():
    rows = [r for r in golden("paper_first_level.txt") if r[0] == "default_private"][0][1:]
    expected = [8 * int(a) + int(b) for a, b in (t.split(",") for t in rows)]
    zz = oracle.zigzag()
    assert list(zz[:6]) == expected


def test_zigzag_is_antidiagonal_permutation():
    zz = oracle.zigzag()
    assert sorted(zz.tolist()) == list(range(64))
    s = [(n // 8) + (n % 8) for n in zz]
    assert s == sorted(s)
    # alternating direction: on odd diagonals the row index increases
    for d in range(15):
        rows = [n // 8 for n in zz if (n // 8) + (n % 8) == d]
        assert rows == (sorted(rows) if d % 2 == 1 else sorted(rows, reverse=True))


def test_value_ranges_from_report():
    fx = {r[0]: r[1:] for r in golden("paper_first_level.txt")}
    dc_max = float(fx["dc_max"][0])
    ac_bits = int(fx["ac_abs_max_bits"][0])
    B = oracle.basis()
    # all-255 block: DC is exactly the bound; all-zero block: 0
    C = oracle.dct_blocks(np.full((1, 8, 8), 255, np.uint8))[0]
    assert abs(C[0] - dc_max) < 1e-9
    # the extreme of each AC coefficient over uint8 blocks is attained at
    # x = 255 * [B_n > 0] (a linear function over a box); check all 63 fit sign + 10 bits
    worst = 0.0
    for n in range(1, 64):
        x = (255 * (B[n] > 0)).astype(np.uint8).reshape(1, 8, 8)
        c = oracle.dct_blocks(x)[0, n]
        worst = max(worst, abs(c))
    assert worst <= 2 ** ac_bits - 1 + 1e-9
    assert abs(worst - 1020.0) < 1e-9


def test_q2_table_matches_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    T = oracle.q2_table()
    pi = mpmath.pi
    margin = mpmath.mpf(1)
    for u in range(8):
        for v in range(8):
            for y in range(8):
                for x in range(8):
                    cu = mpmath.sqrt(mpmath.mpf(1) / 8) if u == 0 else mpmath.mpf(1) / 2
                    cv = mpmath.sqrt(mpmath.mpf(1) / 8) if v == 0 else mpmath.mpf(1) / 2
                    val = cu * cv * mpmath.cos((2 * y + 1) * u * pi / 16) * mpmath.cos((2 * x + 1) * v * pi / 16) * 2 ** 20
                    r = int(mpmath.nint(val))
                    frac = abs(val - mpmath.floor(val) - mpmath.mpf(1) / 2)
                    margin = min(margin, frac)
                    assert T[8 * u + v, 8 * y + x] == r
    # no entry sits near a rounding tie, so the FP64 table is unambiguous
    # (exact multiples of 2^17 have frac = 1/2 and are integers already)
    assert margin > 1e-6 or margin == mpmath.mpf(1) / 2


def _round_half_even_fraction(num, den):
    """Python integer round-half-even of num/den (den > 0), brute-force reference."""
    q, r = divmod(num, den)
    if 2 * r > den or (2 * r == den and q % 2 == 1):
        q += 1
    return q


def test_q2_matches_integer_definition_and_bounds():
    rng = np.random.default_rng(5)
    pix = rng.integers(0, 256, size=(1, 64, 64), dtype=np.uint8)
    # add structured blocks: constant, checkerboard, extremes, tie patterns
    pix[0, :8, :8] = 255
    pix[0, :8, 8:16] = (np.indices((8, 8)).sum(0) % 2 * 255).astype(np.uint8)
    pix[0, 8:16, :8] = 0
    pix[0, 8:16, 8:16] = 0
    pix[0, 8, 8] = 2
    pix[0, 11, 11] = 2           # C(1,1) = 0.5 exactly: an exact tie of the real coefficient
    nat = oracle.zigzag()[:10]
    q = oracle.q2_blocks(pix, nat)
    T = oracle.q2_table().astype(object)
    X = oracle.blocks_of(pix).astype(object)
    C = oracle.dct_blocks(pix)
    B = oracle.basis()
    for b in range(X.shape[0]):
        for l, n in enumerate(nat):
            acc = sum(X[b, p] * T[n, p] for p in range(64))
            assert q[b, l] == _round_half_even_fraction(acc, 1 << 20)
            bound = 0.5 + 255 * np.abs(T[n].astype(np.float64) / 2 ** 20 - B[n]).sum()
            assert abs(q[b, l] - C[b, n]) <= bound + 1e-12
    # DC closed form: round half to even of S/8
    S = oracle.blocks_of(pix).astype(np.int64).sum(1)
    assert np.array_equal(q[:, 0], np.array([_round_half_even_fraction(int(s), 8) for s in S]))
    # tie block: X[0,0] = X[3,3] = 2 -> C(1,1) = 0.5; record the integer rule's decision
    b_tie = 1 * 8 + 1  # block (by=1, bx=1) of the 64x64 plane
    l11 = list(nat).index(9)
    assert abs(C[b_tie, 9] - 0.5) < 1e-12
    assert q[b_tie, l11] in (0, 1)
