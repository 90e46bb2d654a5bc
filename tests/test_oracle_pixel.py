"""Pins of the pixel-domain fragment oracle (oracle/pixel.py): the report's
11-bit private storage (Sec. 6.4.3), the public part as the inverse DCT of
the remaining coefficients stored as bytes (Sec. 6.3.1-6.3.2), the strong
level's SHA-512 mask (Sec. 6.3.2, Fig. 8) and its statistical effect
(Sec. 6.6)."""
import hashlib

import numpy as np
import pytest

import oracle
import synth
from oracle import pixel as px


def _adversarial():
    rng = np.random.default_rng(11)
    blocks = [np.zeros((8, 8)), np.full((8, 8), 255), np.indices((8, 8)).sum(0) % 2 * 255,
              (np.indices((8, 8))[1] >= 4) * 255, rng.integers(0, 256, (8, 8)), np.full((8, 8), 128),
              (np.indices((8, 8))[0] * 36.4).round()]
    row = np.concatenate([b.astype(np.uint8) for b in blocks] + [np.zeros((8, 8), np.uint8)], axis=1)
    return row[None]


def test_11_bit_fields_hand_example():
    # DC 2040 unsigned in 11 bits, AC -1 as sign bit + magnitude 1 (Sec. 6.4.3):
    # fields 0x7F8 | 0x401 << 11 = 0x200FF8, little-endian bit stream
    q = np.array([[2040, -1]])
    assert px.pack11(q, 0b11).tolist() == [0xF8, 0x0F, 0x20]
    # AC-only selection: +1020 and -1020
    q = np.array([[1020, -1020]])
    v = 1020 | ((1024 | 1020) << 11)
    assert px.pack11(q, 0b110).tolist() == [v & 0xFF, (v >> 8) & 0xFF, (v >> 16) & 0xFF]


def test_storage_fraction_matches_the_report():
    # 11 bits x 6 coefficients per 64 samples = 12.9 % of the image (Sec. 6.4.3)
    pub, priv = px.fragment_bytes(1, 4096, 4096, oracle.prefix_mask(5))
    assert pub == 4096 * 4096
    assert round(100 * priv / (4096 * 4096), 1) == 12.9
    assert px.tile_stride(6) == 88 * 6 and px.tile_stride(5) == 448   # 440 rounded up to 16
    assert px.private_bytes(65, 5) == 448 + 7                           # last tile: 55 bits


@pytest.mark.parametrize("mask", [1, 0b11, oracle.prefix_mask(5), oracle.prefix_mask(9), 0b10110100110,
                                  (1 << 16) - 2])
def test_pack_round_trip(mask):
    rng = np.random.default_rng(mask)
    P = oracle.popcount(mask)
    nb = 200
    q = rng.integers(-1020, 1021, (nb, P))
    if mask & 1:
        q[:, 0] = rng.integers(0, 2041, nb)
    assert np.array_equal(px.unpack11(px.pack11(q, mask), nb, mask), q)


def test_inverse_table_closed_forms():
    Bi = px.inv_table()
    assert np.all(Bi[0] == 8192)                              # 2^16 / 8
    # u = v = 4: entries +-1/8 exactly
    assert np.all(np.abs(Bi[36]) == 8192)
    # orthogonality up to the rounding of the entries (|e| <= 1/2 each)
    G = Bi @ Bi.T
    off = np.abs(G - np.diag(np.diag(G))).max()
    assert off <= 64 * 2 ** 15 and np.abs(np.diag(G) - 2 ** 32).max() <= 64 * 2 ** 16


def test_rhe_shift_ties_and_signs():
    a = np.array([3 * 2 ** 15, 2 ** 15, -(2 ** 15), -3 * 2 ** 15, 2 ** 15 + 1, -(2 ** 15) - 1, 5, -5])
    assert px.rhe_shift(a, 16).tolist() == [2, 0, 0, -2, 1, -1, 0, 0]


def test_dc_only_reconstruction_is_the_block_mean():
    pix = _adversarial()
    q = px.private_ints(pix, 1)
    R = px.recon_private(q, 1)
    blk = oracle.blocks_of(pix).astype(np.int64)
    s = blk.sum(1)
    # q = rhe(S / 8), R = floor(q / 8 + 1/2) at every sample
    assert np.array_equal(q[:, 0], px.rhe_shift(s, 3))
    assert np.array_equal(R, np.repeat(np.floor(q[:, 0] / 8 + 0.5).astype(np.int64)[:, None], 64, 1))


@pytest.mark.parametrize("mask", [oracle.prefix_mask(2), oracle.prefix_mask(5), oracle.prefix_mask(9)])
def test_public_is_the_inverse_dct_of_the_rest(mask):
    # P (mod 256) against the report's definition IDCT(C with private zeroed),
    # computed independently in FP64; |P - IDCT(rest)| = |R - IDCT(C_priv)|
    # <= 1/2 + sum |q| 2^-17 + |sum_j (q_j - C_j) B_j(p)|
    pix = np.concatenate([_adversarial()[:, :, :64], synth.image(8, 64, 1, 1, 3).numpy()], axis=2)
    out = px.frag(pix, mask)
    zpos, nat = px.private_positions(mask)
    C = oracle.dct_blocks(pix)
    rest = C.copy()
    rest[:, nat] = 0.0
    want = oracle.idct_blocks(rest)
    got = oracle.blocks_of(out["public"]).astype(np.float64)
    diff = (got - want + 128.0) % 256.0 - 128.0               # circular difference
    q = out["q"].astype(np.float64)
    B = oracle.basis()
    bound = 0.5 + np.abs(q).sum(1, keepdims=True) * 2.0 ** -17 + np.abs((q - C[:, nat]) @ B[nat]) + 1e-9
    assert np.all(np.abs(diff) <= bound)


@pytest.mark.parametrize("strong", [False, True])
@pytest.mark.parametrize("mask", [1, oracle.prefix_mask(5), oracle.prefix_mask(9), 0b1011000100101110, (1 << 16) - 2])
def test_round_trip_exact(mask, strong):
    pix = np.concatenate([_adversarial(), synth.image(8, 64, 1, 1, 4).numpy()], axis=2)
    key, c0 = synth.aes_key(1), synth.ctr0(1, 4)
    out = px.frag(pix, mask, strong, key, c0)
    back = px.defrag(pix.shape, mask, out["public"], strong=strong, key=key, ctr0=c0, cipher=out["cipher"])
    assert np.array_equal(back, pix)
    assert np.array_equal(oracle.ctr_xor(key, c0, out["cipher"]), out["private"])


def test_strong_keystream_fips_vector():
    # FIPS 180-2 SHA-512 example (two-block message of 896 bits): 56 int16
    # little-endian values whose bytes spell the message
    msg = (b"abcdefghbcdefghicdefghijdefghijkefghijklfghijklmghijklmn"
           b"hijklmnoijklmnopjklmnopqklmnopqrlmnopqrsmnopqrstnopqrstu")
    q = np.frombuffer(msg, "<i2").astype(np.int64)[None]
    want = bytes.fromhex("8e959b75dae313da8cf4f72814fc143f8f7779c6eb9f7fa17299aeadb6889018"
                         "501d289e4900f7e4331b99dec4b5433ac7d329eeb6dd26545e96e55b874be909")
    assert px.strong_keystream(q)[0].tobytes() == want


def test_strong_mask_depends_only_on_the_private_integers():
    pix = synth.image(16, 64, 1, 1, 5).numpy()
    mask = oracle.prefix_mask(5)
    weak = px.frag(pix, mask)
    strong = px.frag(pix, mask, strong=True)
    ks = oracle.blocks_of(weak["public"]) ^ oracle.blocks_of(strong["public"])
    q = weak["q"]
    assert np.array_equal(ks, px.strong_keystream(q))
    # two blocks with equal private integers get equal masks, different ones differ
    q2 = np.stack([q[0], q[0], q[1]])
    k2 = px.strong_keystream(q2)
    assert np.array_equal(k2[0], k2[1]) and not np.array_equal(k2[0], k2[2])
    assert k2[0].tobytes() == hashlib.sha512(q[0].astype("<i2").tobytes()).digest()


def test_strong_level_statistics_of_the_report():
    # Sec. 6.6: the strong-level public image has a flat histogram and no
    # correlation between adjacent samples; the first-level public is neither
    pix = synth.image(512, 512, 1, 1).numpy()
    mask = oracle.prefix_mask(5)
    weak = px.frag(pix, mask)["public"][0].astype(np.float64)
    strong = px.frag(pix, mask, strong=True)["public"][0].astype(np.float64)
    n = strong.size
    h = np.bincount(strong.astype(np.int64).ravel(), minlength=256)
    chi2 = ((h - n / 256) ** 2 / (n / 256)).sum()
    hw = np.bincount(weak.astype(np.int64).ravel(), minlength=256)
    chi2w = ((hw - n / 256) ** 2 / (n / 256)).sum()
    assert chi2 < 255 + 8 * np.sqrt(2 * 255) and chi2w > 100 * 255
    r_strong = np.corrcoef(strong[:, :-1].ravel(), strong[:, 1:].ravel())[0, 1]
    r_orig = np.corrcoef(pix[0][:, :-1].ravel().astype(float), pix[0][:, 1:].ravel().astype(float))[0, 1]
    assert abs(r_strong) < 0.01 and r_orig > 0.5


def test_8bit_storage_fraction_matches_the_report():
    # Sec. 6.4.3: DC in 11 bits and 5 AC in 8 bits = 5/64 + 11/8/64 = 9.96 % of the image
    mask = oracle.prefix_mask(5)
    assert px.record_bits(mask, 7) == 11 + 5 * 8
    assert round(100 * px.record_bits(mask, 7) / 512, 2) == 9.96
    # tiles start on AES-block boundaries: 64 records of 51 bits are 408 bytes,
    # padded to 416 (the stored fragment is 10.16 % of the image)
    assert px.tile_stride(6, 51) == 416
    _, priv = px.fragment_bytes(1, 4096, 4096, mask, ac_bits=7)
    assert priv == 4095 * 416 + 408  # the last tile is not padded


def test_8bit_fields_hand_example_and_clamping():
    # DC 2040 in 11 bits; AC -200 clamps to -127: sign bit 7 above magnitude 127
    q = np.array([[2040, -200]])
    v = 0x7F8 | ((0x80 | 127) << 11)
    assert px.pack11(q, 0b11, ac_bits=7).tolist() == [v & 0xFF, (v >> 8) & 0xFF, (v >> 16) & 0xFF]
    assert px.unpack11(px.pack11(q, 0b11, ac_bits=7), 1, 0b11, ac_bits=7).tolist() == [[2040, -127]]


@pytest.mark.parametrize("strong", [False, True])
def test_8bit_storage_loses_only_clamped_blocks(strong):
    mask = oracle.prefix_mask(5)
    pix = np.concatenate([_adversarial(), synth.image(8, 64, 1, 1, 4).numpy()], axis=2)
    out = px.frag(pix, mask, strong, ac_bits=7)
    back = px.defrag(pix.shape, mask, out["public"], out["private"], strong=strong, ac_bits=7)
    clamped = (np.abs(out["q"][:, 1:]) > 127).any(axis=1)
    same = (oracle.blocks_of(back) == oracle.blocks_of(pix)).all(axis=1)
    assert np.all(same[~clamped]) and clamped.any() and not np.all(same[clamped])
    # a clamped block is off by exactly R(stored) - R(exact), modulo 256
    qs = px.stored_ints(out["q"], mask, 7)
    d = (px.recon_private(qs, mask) - px.recon_private(out["q"], mask)) & 0xFF
    got = (oracle.blocks_of(back).astype(np.int64) - oracle.blocks_of(pix).astype(np.int64)) & 0xFF
    assert np.array_equal(got, d)


def test_8bit_storage_exact_when_no_ac_exceeds_127():
    # a low-contrast image (every private AC within 8-bit storage) comes back exactly
    pix = (synth.image(64, 64, 1, 1, 2).numpy() // 4 + 96).astype(np.uint8)
    mask = oracle.prefix_mask(5)
    out = px.frag(pix, mask, True, ac_bits=7)
    assert np.abs(out["q"][:, 1:]).max() <= 127
    assert np.array_equal(px.defrag(pix.shape, mask, out["public"], out["private"], strong=True, ac_bits=7), pix)
