"""GPU parity of the plain (FP32) form against the CPU oracle, through the C ABI.

Bars: private integers and ciphertext bit-exact; public coefficients within
1e-5 of the FP64 oracle, normwise per block relative to the block's pixel
norm (Parseval: the coefficient vector has the same norm), all-zero blocks
exactly 0; reconstructed pixels bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

sf = pytest.importorskip("paper_1512_02951_amd")

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert sf.lib().sf_init() == 0, sf.lib().sf_last_error()


def _adversarial(C=1):
    rng = np.random.default_rng(11)
    p = rng.integers(0, 256, size=(C, 64, 64), dtype=np.uint8)
    yy, xx = np.indices((8, 8))
    blocks = [np.zeros((8, 8)), np.full((8, 8), 255), (yy + xx) % 2 * 255, (xx % 2) * 255, (yy % 2) * 255,
              (xx >= 4) * 255, (yy >= 4) * 255, ((yy >= 4) ^ (xx >= 4)) * 255, np.full((8, 8), 4),
              np.full((8, 8), 128)]
    for i, b in enumerate(blocks):
        p[0, 8 * (i // 8):8 * (i // 8) + 8, 8 * (i % 8):8 * (i % 8) + 8] = b
    return p


def _check(x, mask, key=None, ctr0=None, label="", per_tile=4096):
    """Round trip through the C ABI and compare with the oracle.  Small test
    images get the largest exception capacity (every sample of a tile), so
    even selections with almost all coefficients private fit."""
    print("case:", label, x.shape, hex(mask), flush=True)
    C, H, W = x.shape
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pb, qb, _ = sf.fragment_sizes(H, W, C, mask)
    out = sf.Fragments(torch.empty(max(pb // 4, 1), dtype=torch.float32, device="cuda"),
                       torch.empty(max(qb, 16), dtype=torch.uint8, device="cuda"),
                       sf.ExceptionList.empty((C, H, W), mask, per_tile=per_tile), None, (C, H, W), mask, "fp32")
    fr = sf.frag_image(xd, mask, key, ctr0, out=out, status=status)
    y = sf.defrag_image(fr, key, ctr0, status=status)
    torch.cuda.synchronize()
    ref = oracle.frag(x, mask, key, ctr0)
    nb, npriv = ref["nb"], ref["npriv"]
    npub = 64 - npriv
    # private fragment: bit-exact
    got_priv = fr.private.cpu().numpy()[: 2 * nb * npriv]
    if key is None:
        assert np.array_equal(got_priv.view("<i2"), ref["private"]), "private integers differ"
    else:
        assert np.array_equal(got_priv, ref["cipher"]), "ciphertext differs"
    # public fragment: normwise per block
    if npub:
        pub = oracle.tile_unpack(fr.public.cpu().numpy()[: nb * npub].astype(np.float64), nb, npub)
        pub_ref = oracle.tile_unpack(ref["public"], nb, npub)
        nrm = np.linalg.norm(oracle.blocks_of(x).astype(np.float64), axis=1)
        err = np.linalg.norm(pub - pub_ref, axis=1)
        zero = nrm == 0
        assert np.all(err[zero] == 0), "all-zero block not exactly zero"
        rel = err[~zero] / nrm[~zero]
        assert rel.size == 0 or rel.max() <= TOL_FP32, "public rel err %g" % rel.max()
    # reconstruction: bit-exact
    assert int(status.item()) == 0, "status %d" % status.item()
    assert torch.equal(y.cpu(), torch.from_numpy(x)), "round trip differs"
    return fr, ref


def test_workload1_512_gray_k2():
    x = synth.image(512, 512, 1, 1).numpy()
    _check(x, sf.prefix_mask(2), synth.aes_key(1), synth.ctr0(1), "512x512 gray k=2")


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 24, 40), (3, 64, 96), (2, 136, 264), (1, 520, 8)])
@pytest.mark.parametrize("k", [0, 1, 2, 5, 9])
def test_ragged_shapes_prefix_masks(shape, k):
    C, H, W = shape
    x = synth.image(H, W, C, 1, 7).numpy()
    _check(x, sf.prefix_mask(k), synth.aes_key(1), synth.ctr0(1, 7), "ragged")


@pytest.mark.parametrize("mask", [(1 << 21) - 1, (1 << 64) - 1, 0b111110, 0x8000000000000001,
                                  int(np.random.default_rng(3).integers(1, 1 << 62))])
def test_runtime_masks(mask):
    x = np.concatenate([_adversarial(), synth.image(64, 64, 1, 1, 9).numpy()])
    _check(x, mask, synth.aes_key(1), synth.ctr0(1, 9), "runtime mask")


@pytest.mark.parametrize("k", [2, 5, 9, 20])
def test_adversarial_blocks_and_clear_private(k):
    x = _adversarial(2)
    _check(x, sf.prefix_mask(k), None, None, "clear private")
    _check(x, sf.prefix_mask(k), synth.aes_key(1), synth.ctr0(1, 2), "encrypted")


def test_exceptions_are_produced_and_applied():
    # k = 9 on natural-like content needs exceptions (FP64 oracle finds some too)
    x = synth.image(256, 256, 1, 1, 5).numpy()
    fr, ref = _check(x, sf.prefix_mask(9), synth.aes_key(1), synth.ctr0(1, 5), "k=9 exceptions")
    assert ref["exc_index"].size > 0
    idx, val, counts = fr.exceptions.decode()
    assert idx.size > 0
    assert np.array_equal(x.ravel()[idx], val)
    assert len(set(idx.tolist())) == idx.size
    assert counts.sum() == idx.size


def test_no_exception_buffer_needed_for_small_selections():
    x = synth.image(64, 64, 1, 1, 4).numpy()
    for k in range(5):
        assert not sf.exception_bytes(64, 64, 1, sf.prefix_mask(k), 8)[1]
        fr, _ = _check(x, sf.prefix_mask(k), synth.aes_key(1), synth.ctr0(1), "no exceptions k=%d" % k)
        assert fr.exceptions.buf is None
    assert sf.exception_bytes(64, 64, 1, sf.prefix_mask(5), 8)[1]


def test_exception_overflow_sets_status():
    x = synth.image(128, 128, 1, 1, 6).numpy()
    xd = torch.from_numpy(x).cuda()
    mask = (1 << 40) - 1
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pb, qb, _ = sf.fragment_sizes(128, 128, 1, mask)
    fr = sf.Fragments(torch.empty(pb // 4, dtype=torch.float32, device="cuda"),
                      torch.empty(qb, dtype=torch.uint8, device="cuda"),
                      sf.ExceptionList.empty((1, 128, 128), mask, per_tile=4096), None, (1, 128, 128), mask, "fp32")
    sf.frag_image(xd, mask, None, None, out=fr, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    _, _, counts = fr.exceptions.decode()
    assert counts.max() > 1
    small = sf.ExceptionList.empty(fr.shape, mask, per_tile=1)
    fr2 = sf.Fragments(fr.public, fr.private, small, None, fr.shape, mask, "fp32")
    sf.frag_image(xd, mask, None, None, out=fr2, status=status)
    torch.cuda.synchronize()
    _, _, counts2 = small.decode()
    assert np.array_equal(counts, counts2)
    assert int(status.item()) & sf.SF_STATUS_EXC_OVERFLOW


@pytest.mark.parametrize("nbytes", [1, 15, 16, 17, 1000, 4096 + 5, 1 << 20])
@pytest.mark.parametrize("first", [0, 3])
def test_encrypt_private_matches_oracle(nbytes, first):
    rng = np.random.default_rng(nbytes + first)
    key = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
    ctr0 = bytes(7) + b"\x02" + b"\xff" * 7 + b"\xfe"  # carries through the low 64 bits
    data = rng.integers(0, 256, nbytes, dtype=np.uint8)
    d = torch.from_numpy(data).cuda()
    out = sf.encrypt_private(key, ctr0, d, first_block=first)
    ref = oracle.ctr_xor(key, ctr0, data, first_block=first)
    assert np.array_equal(out.cpu().numpy(), ref)
    sf.encrypt_private(key, ctr0, out, out=out, first_block=first)  # in place, decrypt
    assert np.array_equal(out.cpu().numpy(), data)


def test_published_ctr_vector_on_gpu():
    from conftest import golden
    rows = golden("sp800_38a_ctr_aes128.txt")
    key = bytes.fromhex([r for r in rows if r[0] == "key"][0][1])
    ctr0 = bytes.fromhex([r for r in rows if r[0] == "ctr0"][0][1])
    pt = b"".join(bytes.fromhex(r[1]) for r in rows if r[0] == "block")
    ct = b"".join(bytes.fromhex(r[2]) for r in rows if r[0] == "block")
    d = torch.frombuffer(bytearray(pt), dtype=torch.uint8).cuda()
    assert sf.encrypt_private(key, ctr0, d).cpu().numpy().tobytes() == ct


def test_determinism():
    x = synth.image(256, 320, 3, 1, 8).cuda()
    key, ctr0 = synth.aes_key(1), synth.ctr0(1, 8)
    a = sf.frag_image(x, sf.prefix_mask(5), key, ctr0)
    b = sf.frag_image(x, sf.prefix_mask(5), key, ctr0)
    torch.cuda.synchronize()
    assert torch.equal(a.public.view(torch.int32), b.public.view(torch.int32))
    assert torch.equal(a.private, b.private)
    assert torch.equal(a.exceptions.buf, b.exceptions.buf)


def test_workload2_full_size_4096_rgb_k5():
    """The throughput workload at full size, every fragment compared with the oracle."""
    print("case: 4096x4096x3 k=5 full size", flush=True)
    x = synth.image(4096, 4096, 3, 2, 0, device="cuda")
    key, ctr0 = synth.aes_key(2), synth.ctr0(2, 0)
    mask = sf.prefix_mask(5)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    fr = sf.frag_image(x, mask, key, ctr0, status=status)
    y = sf.defrag_image(fr, key, ctr0, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(x, y)
    xh = x.cpu().numpy()
    ref = oracle.frag(xh, mask, key, ctr0)
    assert np.array_equal(fr.private.cpu().numpy(), ref["cipher"])
    nb = ref["nb"]
    pub = fr.public.cpu().numpy().astype(np.float64)
    # tile layout is a permutation of (block, coefficient): compare per block
    diff = oracle.tile_unpack(pub - ref["public"], nb, 58)
    nrm = np.linalg.norm(oracle.blocks_of(xh).astype(np.float64), axis=1)
    err = np.linalg.norm(diff, axis=1)
    zero = nrm == 0
    assert np.all(err[zero] == 0), "all-zero block not exactly zero"
    rel = err[~zero] / nrm[~zero]
    print("public max rel err %.3e, zero blocks %d, gpu exceptions %d, oracle fp64 exceptions %d"
          % (rel.max(), int(zero.sum()), int(fr.exceptions.decode()[2].sum()), ref["exc_index"].size), flush=True)
    assert rel.max() <= TOL_FP32
