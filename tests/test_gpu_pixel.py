"""GPU parity of the pixel-domain formats (11-bit private fields, byte public
part, SHA-512 strong level) against the oracle, through the C ABI.  Integer
work: public bytes, packed private bytes (plaintext and ciphertext) and the
restored image must be bit-identical to the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import pixel as opx

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import pixel  # noqa: E402

pytestmark = pytest.mark.gpu


def _adversarial():
    rng = np.random.default_rng(11)
    blocks = [np.zeros((8, 8)), np.full((8, 8), 255), np.indices((8, 8)).sum(0) % 2 * 255,
              (np.indices((8, 8))[1] >= 4) * 255, rng.integers(0, 256, (8, 8)), np.full((8, 8), 128),
              (np.indices((8, 8))[0] * 36.4).round(), np.indices((8, 8))[1] % 2 * 255]
    return np.concatenate([b.astype(np.uint8) for b in blocks], axis=1)[None]


def _check(x, mask, strong, key=None, ctr0=None, label="", storage_bits=11):
    print("case:", label, x.shape, hex(mask), strong, key is not None, storage_bits, flush=True)
    ac_bits = 10 if storage_bits == 11 else 7
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    fr = pixel.pixel_frag_image(xd, mask, strong, key, ctr0, storage_bits=storage_bits)
    y = pixel.pixel_defrag_image(fr, key, ctr0)
    torch.cuda.synchronize()
    ref = opx.frag(x, mask, strong, key, ctr0, ac_bits=ac_bits)
    assert np.array_equal(fr.public.cpu().numpy(), ref["public"]), "public bytes differ"
    n = ref["private"].size
    assert pixel.fragment_sizes(*x.shape[1:], x.shape[0], mask, strong, storage_bits)[1] == n
    want = ref["cipher"] if key is not None else ref["private"]
    assert np.array_equal(fr.private.cpu().numpy()[:n], want), "private bytes differ"
    back = opx.defrag(x.shape, mask, ref["public"], ref["private"], strong=strong, ac_bits=ac_bits)
    assert np.array_equal(y.cpu().numpy(), back), "restored image differs from the oracle's"
    if storage_bits == 11:
        assert torch.equal(y.cpu(), torch.from_numpy(x)), "round trip differs"


MASKS = [1, 0x7, 0x3f, 0x3ff, 0b1011000100101110, (1 << 16) - 2, (1 << 16) - 1, 0b11]


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("strong", [False, True])
def test_masks_adversarial_and_synthetic(mask, strong):
    x = np.concatenate([_adversarial(), synth.image(8, 64, 1, 1, 6).numpy()], axis=2)
    _check(x, mask, strong, synth.aes_key(1), synth.ctr0(1, 6), "masks")


@pytest.mark.parametrize("mask", [0x7, 0x3f, 0x3ff, (1 << 16) - 2, 0b1011000100101110])
@pytest.mark.parametrize("strong", [False, True])
def test_8bit_storage(mask, strong):
    # the report's lossy storage: bit-exact against the oracle, including the
    # restored image (exact except where an AC was clamped)
    x = np.concatenate([_adversarial(), synth.image(8, 64, 1, 1, 6).numpy()], axis=2)
    _check(x, mask, strong, synth.aes_key(1), synth.ctr0(1, 6), "8-bit", storage_bits=8)
    _check(synth.image(72, 136, 3, 2, 5).numpy(), mask, strong, None, None, "8-bit ragged", storage_bits=8)


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 24, 40), (1, 72, 136), (2, 64, 512), (1, 8, 4104)])
@pytest.mark.parametrize("mask", [0x3f, 0x1f])
def test_shapes_and_ragged_tiles(shape, mask):
    C, H, W = shape
    x = synth.image(H, W, C, 2, 3).numpy()
    _check(x, mask, True, synth.aes_key(2), synth.ctr0(2, 3), "shapes")
    _check(x, mask, False, None, None, "shapes plain")


def test_full_size_4096_rgb_strong():
    H = W = 4096
    C = 3
    mask = sf.prefix_mask(5)
    key, c0 = synth.aes_key(2), synth.ctr0(2, 0)
    x = synth.image(H, W, C, 2, 0, device="cuda")
    fr = pixel.pixel_frag_image(x, mask, True, key, c0)
    y = pixel.pixel_defrag_image(fr, key, c0)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    _, qb = pixel.fragment_sizes(H, W, C, mask)
    assert qb == opx.fragment_bytes(C, H, W, mask)[1]
    # sampled tiles: whole tiles of the oracle (every block of the tile)
    nb = C * H * W // 64
    ntiles = nb // 64
    rng = np.random.default_rng(7)
    tiles = np.sort(rng.choice(ntiles, 24, replace=False))
    xb = x.view(C, H // 8, 8, W // 8, 8).permute(0, 1, 3, 2, 4).reshape(nb, 64).cpu().numpy()
    pub = fr.public.view(C, H // 8, 8, W // 8, 8).permute(0, 1, 3, 2, 4).reshape(nb, 64).cpu().numpy()
    plain = oracle.ctr_xor(key, c0, fr.private.cpu().numpy()[:qb])
    st = opx.tile_stride(6)
    for t in tiles:
        blk = xb[64 * t:64 * t + 64]
        img = blk.reshape(64, 8, 8).transpose(1, 0, 2).reshape(1, 8, 512)  # the 64 blocks side by side
        ref = opx.frag(img, mask, True)
        assert np.array_equal(oracle.blocks_of(ref["public"]), pub[64 * t:64 * t + 64])
        assert np.array_equal(ref["private"], plain[t * st:(t + 1) * st])


def test_errors():
    x = torch.zeros((1, 16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SefragError) as e:
        pixel.pixel_frag_image(x, (1 << 17) - 1)
    assert e.value.code == sf.SF_ERANGE
    with pytest.raises(sf.SefragError) as e:
        pixel.pixel_frag_image(torch.zeros((1, 12, 16), dtype=torch.uint8, device="cuda"), 0x3f)
    assert e.value.code == sf.SF_ESHAPE
    assert pixel.fragment_sizes(16, 16, 1, 0x3f) == (256, 33)
    assert pixel.fragment_sizes(16, 16, 1, 0x3f, storage_bits=8) == (256, (51 * 4 + 7) // 8)
