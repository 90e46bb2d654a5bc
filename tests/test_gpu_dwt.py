"""GPU parity of the wavelet variant (LeGall 5/3, two levels on 8x8 blocks)
against the integer oracle, through the C ABI.  Integer work: public and
private fragments, ciphertext and the restored samples must all be
bit-identical to the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import dwt as odwt

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import dwt  # noqa: E402

pytestmark = pytest.mark.gpu


def _check(x, key=None, ctr0=None, label=""):
    print("case:", label, x.shape, key is not None, flush=True)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    fr = dwt.dwt_frag_image(xd, key, ctr0)
    y = dwt.dwt_defrag_image(fr, key, ctr0)
    torch.cuda.synchronize()
    ref = odwt.frag(x, key, ctr0)
    nb = ref["nb"]
    assert np.array_equal(fr.public.cpu().numpy()[:60 * nb], ref["public"]), "public coefficients differ"
    got = fr.private.cpu().numpy()[:8 * nb]
    if key is None:
        assert np.array_equal(got.view("<i2"), ref["private"]), "private coefficients differ"
    else:
        assert np.array_equal(got, ref["cipher"]), "ciphertext differs"
    assert torch.equal(y.cpu(), torch.from_numpy(x)), "round trip differs"


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 24, 40), (1, 72, 136), (2, 64, 512), (1, 8, 4104)])
@pytest.mark.parametrize("keyed", [False, True])
def test_shapes(shape, keyed):
    C, H, W = shape
    x = synth.image(H, W, C, 2, 3).numpy()
    key, c0 = (synth.aes_key(2), synth.ctr0(2, 3)) if keyed else (None, None)
    _check(x, key, c0, "shapes")


def test_adversarial_blocks():
    x = np.zeros((1, 64, 128), np.uint8)
    x[0, :8, :8] = 255
    x[0, 8:16, 8:16] = (np.indices((8, 8)).sum(0) % 2 * 255).astype(np.uint8)
    x[0, 16:24] = np.random.default_rng(3).integers(0, 256, size=(8, 128), dtype=np.uint8)
    x[0, 24:32] = (np.indices((8, 128)).sum(0) % 2 * 255).astype(np.uint8)
    _check(x, synth.aes_key(2), synth.ctr0(2, 4), "adversarial")


def test_arbitrary_bytes_as_a_gray_image():
    # data-agnostic chunking: any byte string viewed as a W-wide gray image
    data = np.random.default_rng(5).integers(0, 256, size=1024 * 1024, dtype=np.uint8)
    _check(data.reshape(1, 1024, 1024), synth.aes_key(2), synth.ctr0(2, 5), "bytes")


def test_full_size_4096_rgb():
    H = W = 4096
    C = 3
    key, c0 = synth.aes_key(2), synth.ctr0(2, 0)
    x = synth.image(H, W, C, 2, 0, device="cuda")
    fr = dwt.dwt_frag_image(x, key, c0)
    y = dwt.dwt_defrag_image(fr, key, c0)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    # sampled blocks against the oracle (public values and private plaintext)
    nb = C * H * W // 64
    rng = np.random.default_rng(6)
    blocks = np.sort(rng.choice(nb, 4096, replace=False))
    xb = x.view(C, H // 8, 8, W // 8, 8).permute(0, 1, 3, 2, 4).reshape(nb, 64)[torch.from_numpy(blocks).cuda()]
    coef = odwt.dwt_blocks(xb.cpu().numpy())
    pub = fr.public.cpu().numpy()
    pos_pub = oracle.tile_offsets(nb, 60, blocks[:, None], np.arange(60)[None, :])
    want_pub = np.stack([coef[:, r, q] for r, q in odwt.PUBLIC_POS], axis=1)
    assert np.array_equal(pub[pos_pub], want_pub)
    plain = oracle.ctr_xor(key, c0, fr.private.cpu().numpy()[:8 * nb]).view("<i2")
    pos_priv = oracle.tile_offsets(nb, 4, blocks[:, None], np.arange(4)[None, :])
    want_priv = np.stack([coef[:, r, q] for r, q in odwt.PRIVATE_POS], axis=1)
    assert np.array_equal(plain[pos_priv], want_priv)


def test_errors():
    x = torch.zeros((1, 12, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SefragError) as e:
        dwt.dwt_frag_image(x)
    assert e.value.code == sf.SF_ESHAPE
    assert dwt.fragment_sizes(16, 16, 1) == (2 * 60 * 4, 2 * 4 * 4)
