"""Pins for the oracle's whole frag/defrag pipeline (Sec. 6.3.1, Fig. 6; Sec. 5.2, Fig. 3)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import golden


def _adversarial_plane():
    """64x64 plane of hand-made blocks: extremes, checkerboards, stripes, ties."""
    rng = np.random.default_rng(11)
    p = rng.integers(0, 256, size=(64, 64), dtype=np.uint8)
    yy, xx = np.indices((8, 8))
    blocks = [
        np.zeros((8, 8)), np.full((8, 8), 255), (yy + xx) % 2 * 255, (xx % 2) * 255, (yy % 2) * 255,
        (xx >= 4) * 255, (yy >= 4) * 255, ((yy >= 4) ^ (xx >= 4)) * 255, np.full((8, 8), 4),
    ]
    for i, b in enumerate(blocks):
        p[8 * (i // 8):8 * (i // 8) + 8, 8 * (i % 8):8 * (i % 8) + 8] = b
    return p[None]


def test_tile_layout_small_example():
    # 70 blocks, 2 values per block: tile 0 has 64 blocks, tile 1 has 6.
    nb, P = 70, 2
    assert oracle.tile_offset(nb, P, 0, 0) == 0
    assert oracle.tile_offset(nb, P, 5, 0) == 5
    assert oracle.tile_offset(nb, P, 5, 1) == 64 + 5
    assert oracle.tile_offset(nb, P, 64, 0) == 128
    assert oracle.tile_offset(nb, P, 66, 1) == 128 + 6 + 2
    offs = sorted(oracle.tile_offset(nb, P, b, j) for b in range(nb) for j in range(P))
    assert offs == list(range(nb * P))
    vals = np.arange(nb * P).reshape(nb, P)
    flat = oracle.tile_pack(vals)
    for b in range(nb):
        for j in range(P):
            assert flat[oracle.tile_offset(nb, P, b, j)] == vals[b, j]
    assert np.array_equal(oracle.tile_unpack(flat, nb, P), vals)


@pytest.mark.parametrize("k", [0, 2, 5, 9])
def test_fragments_are_the_definition(k):
    pix = _adversarial_plane()
    mask = oracle.prefix_mask(k)
    key, ctr0 = synth.aes_key(1), synth.ctr0(1)
    f = oracle.frag(pix, mask, key, ctr0)
    nb = f["nb"]
    zz = oracle.zigzag()
    C = oracle.dct_blocks(pix)
    priv = oracle.tile_unpack(f["private"], nb, k + 1)
    pub = oracle.tile_unpack(f["public"], nb, 63 - k)
    assert np.array_equal(priv, oracle.q2_blocks(pix, zz[:k + 1]))
    assert np.abs(pub - C[:, zz[k + 1:]]).max() < 1e-12
    plain = f["private"].astype("<i2").tobytes()
    assert np.array_equal(f["cipher"], oracle.ctr_xor(key, ctr0, plain))


@pytest.mark.parametrize("k", [0, 1, 2, 5, 9, 20, 63])
def test_round_trip_exact(k):
    pix = np.concatenate([_adversarial_plane(), synth.image(64, 64, 1, 1).numpy()], 0)
    mask = oracle.prefix_mask(k)
    key, ctr0 = synth.aes_key(1), synth.ctr0(1, 3)
    f = oracle.frag(pix, mask, key, ctr0)
    out = oracle.defrag(pix.shape, mask, f["public"], key=key, ctr0=ctr0, cipher=f["cipher"],
                        exc_index=f["exc_index"], exc_value=f["exc_value"])
    assert np.array_equal(out, pix)
    # without the exception list only the listed pixels may differ
    raw = oracle.defrag(pix.shape, mask, f["public"], private=f["private"])
    bad = np.flatnonzero(raw.ravel() != pix.ravel())
    assert np.array_equal(np.sort(bad), np.sort(f["exc_index"]))


def test_no_exceptions_needed_for_k_up_to_4():
    # rounding bound 0.5 * max_p sum_{private} |B_n(p)| (+ 0.0078 from the integer
    # basis) stays below 1/2 for k <= 4, so the report's 11-bit storage is lossless
    # there (Table 5 "Infinite" PSNR).
    B = oracle.basis()
    zz = oracle.zigzag()
    for k in range(5):
        b = 0.5 * np.abs(B[zz[:k + 1]]).sum(0).max()
        assert b < 0.45
    pix = np.concatenate([_adversarial_plane(), synth.image(128, 128, 1, 1, 2).numpy()[:, :64, :64]], 0)
    for k in range(5):
        f = oracle.frag(pix, oracle.prefix_mask(k))
        assert f["exc_index"].size == 0 and f["max_err"] < 0.5


def test_exceptions_are_needed_for_larger_k():
    # For k = 9 the rounding bound exceeds 1/2 and natural-like content produces
    # pixels that do not round back (the report notes DCT cannot guarantee
    # losslessness, Sec. 6.8).
    B = oracle.basis()
    zz = oracle.zigzag()
    assert 0.5 * np.abs(B[zz[:6]]).sum(0).max() > 0.5
    pix = synth.image(256, 256, 1, 1, 5).numpy()
    f = oracle.frag(pix, oracle.prefix_mask(9))
    assert f["exc_index"].size > 0
    assert f["max_err"] < 0.9


def test_energy_claim_dc_plus_five_ac():
    fx = {r[0]: r[1:] for r in golden("paper_first_level.txt")}
    pix = synth.image(256, 256, 1, 1, 0).numpy()
    C = oracle.dct_blocks(pix)
    zz = oracle.zigzag()
    frac = (C[:, zz[:6]] ** 2).sum() / (C ** 2).sum()
    assert frac > float(fx["energy_fraction_min"][0])


def test_storage_fraction_claim():
    fx = {r[0]: r[1:] for r in golden("paper_first_level.txt")}
    assert abs(11 * 6 / 64 / 8 - float(fx["storage_11bit_fraction"][0])) < 1e-12


def test_different_nonce_changes_ciphertext():
    # per-input IV (Sec. 6.10.6)
    pix = synth.image(64, 64, 1, 1).numpy()
    key = synth.aes_key(1)
    a = oracle.frag(pix, oracle.prefix_mask(5), key, synth.ctr0(1, 0))["cipher"]
    b = oracle.frag(pix, oracle.prefix_mask(5), key, synth.ctr0(1, 1))["cipher"]
    assert not np.array_equal(a, b)


def test_vector_tile_offsets_match_scalar_definition():
    for nb, P in ((70, 2), (64, 5), (1, 3), (200, 58)):
        b = np.repeat(np.arange(nb), P)
        j = np.tile(np.arange(P), nb)
        vec = oracle.tile_offsets(nb, P, b, j)
        assert np.array_equal(vec, [oracle.tile_offset(nb, P, int(x), int(y)) for x, y in zip(b, j)])
