"""The largest images the boundary accepts (fewer than 2^32 samples):
C = 4, H = 32760, W = 32768, i.e. 4 293 918 720 samples.  Fragment byte
offsets pass 2^32 here.  Every path round-trips exactly on the GPU; sampled
tiles (the first, the last and random ones) are compared with the oracle,
bit-exact for integers and ciphertext, normwise 1e-5 for FP32 public values."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import dwt as odwt
from oracle import pixel as opx

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import dwt, pixel  # noqa: E402

pytestmark = pytest.mark.gpu

C, H, W = 4, 32760, 32768
NB = C * (H // 8) * (W // 8)
NT = NB // 64
MASK = (1 << 6) - 1  # DC + 5 AC
KEY, CTR0 = synth.aes_key(2), synth.ctr0(2, 9)


@pytest.fixture(scope="module")
def big():
    assert C * H * W < 2 ** 32 and (C * H * W) > 2 ** 32 - 2 ** 21
    print("case: generating", (C, H, W), flush=True)
    x = synth.image(H, W, C, 2, 9, device="cuda")
    yield x
    del x
    torch.cuda.empty_cache()


def _tiles():
    rng = np.random.default_rng(12)
    return [0, NT - 1] + sorted(rng.choice(NT, 10, replace=False).tolist())


def _tile_image(img, t):
    """The 64 blocks of tile t side by side (a tile lies in one block row
    because W / 8 is a multiple of 64): a (1, 8, 512) host image."""
    b0 = 64 * t
    by_all, bx0 = divmod(b0, W // 8)
    c, by = divmod(by_all, H // 8)
    return img[c, 8 * by:8 * by + 8, 8 * bx0:8 * bx0 + 512].cpu().numpy()[None]


def test_plain_form_max_size(big):
    print("case: plain max size", flush=True)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    fr = sf.frag_image(big, MASK, KEY, CTR0, status=status)
    y = sf.defrag_image(fr, KEY, CTR0, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(big, y)
    del y
    for t in _tiles():
        img = _tile_image(big, t)
        ref = oracle.frag(img, MASK)
        cipher = fr.private[768 * t:768 * (t + 1)].cpu().numpy()
        plain = oracle.ctr_xor(KEY, CTR0, cipher, first_block=48 * t).view("<i2")
        assert np.array_equal(plain, ref["private"]), t
        pub = fr.public[64 * 58 * t:64 * 58 * (t + 1)].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(oracle.tile_unpack(pub - ref["public"], 64, 58), axis=1)
        nrm = np.linalg.norm(oracle.blocks_of(img).astype(np.float64), axis=1)
        assert np.all(err <= 1e-5 * np.maximum(nrm, 1e-30)), t
    del fr
    torch.cuda.empty_cache()


def test_pixel_strong_max_size(big):
    print("case: pixel strong max size", flush=True)
    fr = pixel.pixel_frag_image(big, MASK, True, KEY, CTR0)
    y = pixel.pixel_defrag_image(fr, KEY, CTR0)
    torch.cuda.synchronize()
    assert torch.equal(big, y)
    del y
    st = opx.tile_stride(6)
    for t in _tiles():
        img = _tile_image(big, t)
        ref = opx.frag(img, MASK, True)
        assert np.array_equal(_tile_image(fr.public, t), ref["public"]), t
        cipher = fr.private[st * t:st * (t + 1)].cpu().numpy()
        assert np.array_equal(oracle.ctr_xor(KEY, CTR0, cipher, first_block=st * t // 16), ref["private"]), t
    del fr
    torch.cuda.empty_cache()


def test_wavelet_max_size(big):
    print("case: wavelet max size", flush=True)
    fr = dwt.dwt_frag_image(big, KEY, CTR0)
    y = dwt.dwt_defrag_image(fr, KEY, CTR0)
    torch.cuda.synchronize()
    assert torch.equal(big, y)
    del y
    for t in _tiles():
        img = _tile_image(big, t)
        ref = odwt.frag(img)
        assert np.array_equal(fr.public[64 * 60 * t:64 * 60 * (t + 1)].cpu().numpy(), ref["public"]), t
        cipher = fr.private[512 * t:512 * (t + 1)].cpu().numpy()
        plain = oracle.ctr_xor(KEY, CTR0, cipher, first_block=32 * t).view("<i2")
        assert np.array_equal(plain, ref["private"]), t
    del fr
    torch.cuda.empty_cache()
