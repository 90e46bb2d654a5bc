"""GPU parity of the reduced-precision form (fp16 / bf16 MFMA transforms with
2-bit residual codes and exception slots) against the CPU oracle, through the
C ABI.

Bars: private integers and ciphertext bit-exact; public coefficients within
2e-3 of the FP64 oracle, normwise per block relative to the block's pixel
norm (the stored 16-bit values included); reconstructed pixels bit-exact
through the residual codes and the exception slots; every code-2 sample has
an exception holding its value, and no other sample has one.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

sf = pytest.importorskip("paper_1512_02951_amd")

pytestmark = pytest.mark.gpu

TOL_LP = 2e-3
# bf16 keeps 8 significant bits: storing a coefficient alone can move it by
# up to 2^-8 of its value.  When the dominant coefficients (DC first) are
# private, the public part is small next to the block norm and 2e-3 holds;
# when DC itself is public the stored values can only be held to the storage
# bound (plus the transform's own error).
TOL_BF16_DC_PUBLIC = 2.0 ** -8 + 2e-4
# FP32-accumulated MFMA transform: per coefficient |error| <= (basis
# representation error + accumulation error) * sum_p |x_p|, with |B| <= 1/4
# and 64 FP32 accumulations (64 u, u = 2^-24, below 2^-20).  bf16 splits the
# basis into hi + lo (16 significant bits, 2^-16 relative: 2^-18 per unit of
# the L1 norm); fp16 keeps one half-precision basis (11 bits, 2^-12 relative:
# 2^-14).  The bounds below add a factor-two margin.
TRANSFORM_ERR = {"bf16": 2.0 ** -17, "fp16": 2.0 ** -13}


def _round_like(v: np.ndarray, prec: str) -> np.ndarray:
    """Oracle values rounded to the storage type (round to nearest even)."""
    if prec == "fp16":
        return v.astype(np.float16).astype(np.float64)
    return torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()


def _ulp(v: np.ndarray, prec: str) -> np.ndarray:
    mant = 10 if prec == "fp16" else 7
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** -14)))
    return 2.0 ** (e - mant)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert sf.lib().sf_init() == 0, sf.lib().sf_last_error()


def lp_public_index(nb: int, P: int, blocks, j) -> np.ndarray:
    """Element index of public value j of block b in the reduced-precision
    layout (C ABI): tile t = b // 64 of n_t blocks, half h = (b % 64) // 32
    with m_0 = min(32, n_t) and m_1 = n_t - 32 blocks, each half
    [rank][m_h blocks]: 64 t P + h P m_0 + j m_h + b % 32."""
    b = np.asarray(blocks, np.int64)
    j = np.asarray(j, np.int64)
    t, i = b // 64, b % 64
    nt = np.minimum(64, nb - 64 * t)
    h = i // 32
    m0 = np.minimum(32, nt)
    mh = np.where(h == 0, m0, nt - 32)
    return 64 * t * P + h * P * m0 + j * mh + i % 32


def lp_public_unpack(flat: np.ndarray, nb: int, P: int) -> np.ndarray:
    idx = lp_public_index(nb, P, np.repeat(np.arange(nb), P), np.tile(np.arange(P), nb))
    return flat[idx].reshape(nb, P)


def test_lp_public_index_hand_example():
    # 100 blocks, P = 2: tile 0 halves of 32 blocks, tile 1 (36 blocks) halves of 32 and 4
    assert lp_public_index(100, 2, 0, 0) == 0 and lp_public_index(100, 2, 31, 1) == 32 + 31
    assert lp_public_index(100, 2, 32, 0) == 64 and lp_public_index(100, 2, 33, 1) == 64 + 32 + 1
    assert lp_public_index(100, 2, 64, 1) == 128 + 32 and lp_public_index(100, 2, 96, 0) == 128 + 64
    assert lp_public_index(100, 2, 99, 1) == 128 + 64 + 4 + 3
    idx = lp_public_index(100, 2, np.repeat(np.arange(100), 2), np.tile(np.arange(2), 100))
    assert np.array_equal(np.sort(idx), np.arange(200))


def _public_f64(t: torch.Tensor) -> np.ndarray:
    return t.float().cpu().numpy().astype(np.float64)


def _check(x, mask, prec, key=None, ctr0=None, label=""):
    print("case:", label, prec, x.shape, hex(mask), flush=True)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    fr = sf.frag_image(xd, mask, key, ctr0, precision=prec, status=status)
    y = sf.defrag_image(fr, key, ctr0, status=status)
    torch.cuda.synchronize()
    ref = oracle.frag(x, mask, key, ctr0)
    nb, npriv = ref["nb"], ref["npriv"]
    npub = 64 - npriv
    got = fr.private.cpu().numpy()[: 2 * nb * npriv]
    if key is None:
        assert np.array_equal(got.view("<i2"), ref["private"]), "private integers differ"
    else:
        assert np.array_equal(got, ref["cipher"]), "ciphertext differs"
    if npub:
        pub = lp_public_unpack(_public_f64(fr.public[: nb * npub]), nb, npub)
        pub_ref = oracle.tile_unpack(ref["public"], nb, npub)
        nrm = np.linalg.norm(oracle.blocks_of(x).astype(np.float64), axis=1)
        err = np.linalg.norm(pub - pub_ref, axis=1)
        zero = nrm == 0
        assert np.all(err[zero] == 0), "all-zero block not exactly zero"
        rel = err[~zero] / nrm[~zero]
        tol = TOL_LP if (prec == "fp16" or mask & 1) else TOL_BF16_DC_PUBLIC
        assert rel.size == 0 or rel.max() <= tol, "public rel err %g" % rel.max()
        print("  public max normwise rel err %.3e" % (rel.max() if rel.size else 0.0), flush=True)
        # per value: storage rounding (half an ulp) plus the transform's own
        # error, bounded by TRANSFORM_ERR times the block's pixel L1 norm
        l1 = np.abs(oracle.blocks_of(x).astype(np.float64)).sum(axis=1)[:, None]
        bound = 0.5 * _ulp(_round_like(pub_ref, prec), prec) * (1 + 2.0 ** -7) + TRANSFORM_ERR[prec] * l1
        assert np.all(np.abs(pub - pub_ref) <= bound), "stored value beyond rounding + transform bound"
    codes = residual_codes(fr.residual.cpu().numpy(), x.shape)
    ei, ev, counts = fr.exceptions.decode()
    print("  residual nonzero fraction %.3e, escapes %d" % (np.count_nonzero(codes) / codes.size, ei.size), flush=True)
    flat = np.ascontiguousarray(x).reshape(-1)
    assert np.array_equal(np.sort(ei), np.flatnonzero(codes.reshape(-1) == 2)), "escape codes and slots disagree"
    assert np.array_equal(ev, flat[ei]), "exception values differ from the samples"
    # a code of +1 / -1 means the reconstruction rounded to x - 1 / x + 1: in range
    assert not np.any((codes.reshape(-1) == 1) & (flat == 0)) and not np.any((codes.reshape(-1) == 3) & (flat == 255))
    assert int(status.item()) == 0, "status %d" % status.item()
    assert torch.equal(y.cpu(), torch.from_numpy(x)), "round trip differs"
    return fr, ref


def residual_codes(raw: np.ndarray, shape) -> np.ndarray:
    """2-bit residual codes (layout of the C ABI: one 16-byte record per
    block, sample (y, x) at bit 32 (2 (x / 4) + y / 4) + 8 (x % 4) + 2 (y % 4))
    as an array of the image's shape."""
    C, H, W = shape if len(shape) == 3 else (1,) + tuple(shape)
    nb = C * H * W // 64
    words = raw[: 16 * nb].view("<u4").reshape(nb, 4)
    yy, xx = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    bit = 32 * (2 * (xx // 4) + yy // 4) + 8 * (xx % 4) + 2 * (yy % 4)
    blk = (words[:, bit // 32] >> (bit % 32)) & 3  # (nb, 8, 8)
    return blk.reshape(C, H // 8, W // 8, 8, 8).transpose(0, 1, 3, 2, 4).reshape(C, H, W)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape,k", [((1, 64, 64), 9), ((3, 24, 40), 5), ((1, 8, 8), 0), ((2, 136, 264), 9),
                                     ((1, 512, 512), 9), ((1, 64, 64), 63)])
def test_lp_shapes(prec, shape, k):
    C, H, W = shape
    x = synth.image(H, W, C, 3, 1).numpy()
    _check(x, sf.prefix_mask(k), prec, synth.aes_key(3), synth.ctr0(3, 1), "lp")


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("mask", [0b111110, 0x8000000000000001, (1 << 64) - 1])
def test_lp_runtime_masks_and_clear_private(prec, mask):
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, size=(1, 64, 128), dtype=np.uint8)
    x[0, :8, :8] = 255
    x[0, 8:16, :8] = 0
    _check(x, mask, prec, None, None, "lp runtime mask")


# An 8x8 block whose bf16 public part (DC public, zigzag positions 1-5
# private) reconstructs about 1.7 away from some of its samples: found by a
# search over saturated blocks maximising max |IDCT(stored) - x| with bf16
# storage of the public coefficients, so its residual needs the exception
# slots.
ESCAPE_BLOCK = np.array([[255, 0, 255, 0, 255, 255, 0, 0], [0, 255, 0, 0, 0, 0, 255, 0],
                         [255, 255, 255, 255, 255, 255, 0, 0], [255, 0, 0, 255, 255, 255, 255, 255],
                         [255, 255, 255, 255, 0, 0, 255, 0], [255, 0, 255, 255, 0, 0, 0, 0],
                         [0, 255, 255, 255, 255, 255, 255, 255], [255, 255, 0, 0, 0, 0, 255, 255]], np.uint8)


def test_lp_residual_beyond_one_goes_to_the_exception_slots():
    """bf16 with DC public on blocks that reconstruct 1.7 away: their residual
    codes are 2 and the exception slots restore the samples; with too few
    slots the overflow bit is raised."""
    x = np.tile(ESCAPE_BLOCK, (3, 5))[None]  # 15 copies
    x[0, 8:16, 16:24] = np.rot90(ESCAPE_BLOCK)
    mask = 0b111110
    fr, _ = _check(np.ascontiguousarray(x), mask, "bf16", synth.aes_key(3), synth.ctr0(3, 2), "escapes")
    ei, _, counts = fr.exceptions.decode()
    assert ei.size > 0, "no sample needed an exception"
    # the same image with one slot per tile: overflow reported
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    small = sf.Fragments(public=torch.empty_like(fr.public), private=torch.empty_like(fr.private),
                         exceptions=sf.ExceptionList.empty(x.shape, mask, per_tile=1, precision="bf16"),
                         residual=torch.empty_like(fr.residual), shape=fr.shape, mask=mask, precision="bf16")
    sf.frag_image(xd, mask, None, None, precision="bf16", out=small, status=status)
    torch.cuda.synchronize()
    if counts.max() > 1:
        assert int(status.item()) & sf.SF_STATUS_EXC_OVERFLOW
    assert small.exceptions.decode()[2].max() == counts.max()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_lp_workload3_full_size(prec):
    """16 grayscale 8192x8192 images, k = 9: every round trip exact on the GPU,
    2048 sampled blocks per image compared with the oracle."""
    mask = sf.prefix_mask(9)
    key = synth.aes_key(3)
    H = W = 8192
    nb = H * W // 64
    npub, npriv = 54, 10
    x = torch.empty((1, H, W), dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    worst = 0.0
    rng = np.random.default_rng(33)
    for img in range(16):
        print("case: workload 3 image", img, prec, flush=True)
        synth.image(H, W, 1, 3, img, device="cuda", out=x)
        c0 = synth.ctr0(3, img)
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        fr = sf.frag_image(x, mask, key, c0, precision=prec, status=status)
        sf.defrag_image(fr, key, c0, out=y, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert torch.equal(x, y), "image %d round trip differs" % img
        # sampled blocks: oracle on a strip made of those blocks
        blocks = np.sort(rng.choice(nb, 2048, replace=False))
        xb = x[0].view(H // 8, 8, W // 8, 8).permute(0, 2, 1, 3).reshape(nb, 64)[torch.from_numpy(blocks).cuda()]
        xb = xb.cpu().numpy()
        strip = xb.reshape(-1, 8, 8).transpose(1, 0, 2).reshape(8, -1)[None]
        ref = oracle.frag(strip, mask)
        ref_priv = oracle.tile_unpack(ref["private"], blocks.size, npriv)
        ref_pub = oracle.tile_unpack(ref["public"], blocks.size, npub)
        pub_all = fr.public
        priv_all = fr.private.cpu().numpy()
        # decrypt the sampled private values with the oracle keystream
        for j in range(npriv):
            byte = 2 * oracle.tile_offsets(nb, npriv, blocks, j)
            ks = oracle.ctr_keystream(key, c0, byte // 16)
            k0 = ks[np.arange(byte.size), byte % 16]
            k1 = ks[np.arange(byte.size), byte % 16 + 1]
            plain = (priv_all[byte] ^ k0).astype(np.uint16) | ((priv_all[byte + 1] ^ k1).astype(np.uint16) << 8)
            assert np.array_equal(plain.view(np.int16), ref_priv[:, j]), "private coefficient %d differs" % j
        idx = lp_public_index(nb, npub, np.repeat(blocks, npub), np.tile(np.arange(npub), blocks.size))
        got = _public_f64(pub_all[torch.from_numpy(idx).cuda()]).reshape(blocks.size, npub)
        nrm = np.linalg.norm(xb.astype(np.float64), axis=1)
        err = np.linalg.norm(got - ref_pub, axis=1)
        ok = nrm > 0
        assert np.all(err[~ok] == 0)
        rel = err[ok] / nrm[ok]
        worst = max(worst, float(rel.max()))
        assert rel.max() <= TOL_LP
        del fr
    print("workload 3 %s: worst sampled public normwise rel err %.3e" % (prec, worst), flush=True)
