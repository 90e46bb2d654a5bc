"""GPU tests of the batched form: every image of a mixed batch gives exactly the
fragments of the single-image path (itself checked against the oracle in
test_gpu_plain.py), matches the oracle directly on sampled blocks, and
restores bit-exactly; graph replays, the tuner and the 2000-image workload."""
import numpy as np
import pytest
import torch

import oracle
import synth

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd.batch import Batch  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert sf.lib().sf_init() == 0, sf.lib().sf_last_error()


def _mixed(n=24, seed=4):
    rng = np.random.default_rng(seed)
    imgs, masks, ctrs = [], [], []
    for i in range(n):
        H = int(8 * rng.integers(1, 40))
        W = int(8 * rng.integers(1, 60))
        C = int(rng.choice([1, 3]))
        imgs.append(synth.image(H, W, C, 4, 1000 + i).cuda())
        k = int(rng.choice([1, 2, 5, 9]))
        masks.append(sf.prefix_mask(k) if i % 7 else int(rng.integers(1, 1 << 40)))
        ctrs.append(synth.ctr0(4, 1000 + i))
    return imgs, masks, ctrs


def _check_against_single(b, imgs, masks, ctrs, key):
    for i, (x, m, c0) in enumerate(zip(imgs, masks, ctrs)):
        C, H, W = x.shape
        fr = sf.Fragments(torch.empty_like(b.publics[i]), torch.empty_like(b.privates[i]),
                          sf.ExceptionList(torch.zeros_like(b.excs[i]) if b.excs[i] is not None else None,
                                           sf.DEFAULT_PER_TILE, (C, H, W)), None, (C, H, W), m, "fp32")
        sf.frag_image(x, m, key, c0, out=fr)
        torch.cuda.synchronize()
        # the buffers are padded to at least 16 bytes; compare the fragments' bytes
        pb, qb, _ = sf.fragment_sizes(H, W, C, m)
        assert torch.equal(fr.private[:qb], b.privates[i][:qb]), "image %d private differs" % i
        assert torch.equal(fr.public.view(torch.int32)[: pb // 4],
                           b.publics[i].view(torch.int32)[: pb // 4]), "image %d public" % i
        if b.excs[i] is not None:
            ea = sf.ExceptionList(b.excs[i], sf.DEFAULT_PER_TILE, (C, H, W)).decode()
            eb = fr.exceptions.decode()
            assert np.array_equal(ea[2], eb[2])
            assert sorted(zip(ea[0].tolist(), ea[1].tolist())) == sorted(zip(eb[0].tolist(), eb[1].tolist()))
        assert torch.equal(b.restored[i], x), "image %d round trip" % i


def test_mixed_batch_matches_single_image_path_and_oracle():
    imgs, masks, ctrs = _mixed()
    key = synth.aes_key(4)
    b = Batch(imgs, masks, key, ctrs)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.frag(status=status)
    b.defrag(status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    _check_against_single(b, imgs, masks, ctrs, key)
    for i in range(0, len(imgs), 5):  # oracle directly
        x = imgs[i].cpu().numpy()
        ref = oracle.frag(x, masks[i], key, ctrs[i])
        assert np.array_equal(b.privates[i].cpu().numpy()[: ref["cipher"].size], ref["cipher"])


# (tiles_per_grab, workgroups_per_cu[, schedule]): work queue, then static chunks
@pytest.mark.parametrize("tuning", [(1, 1), (4, 2), (16, 0), (1024, 3),
                                    (1, 1, 1), (2, 3, 1), (8, 0, 1), (1024, 2, 1)])
def test_tunings_give_identical_results(tuning):
    imgs, masks, ctrs = _mixed(12, 5)
    key = synth.aes_key(4)
    b = Batch(imgs, masks, key, ctrs)
    b.frag(tuning)
    b.defrag(tuning)
    torch.cuda.synchronize()
    _check_against_single(b, imgs, masks, ctrs, key)


def test_graph_replays_and_autotune(tmp_path):
    imgs, masks, ctrs = _mixed(16, 6)
    key = synth.aes_key(4)
    b = Batch(imgs, masks, key, ctrs)
    tuning, ms = b.autotune(cache=str(tmp_path / "tune.json"))
    assert tuning[2] in (0, 1) and 1 <= tuning[1] <= 3 and ms > 0
    assert tuning[0] in ((4, 8, 16, 32), (1, 2, 4, 8))[tuning[2]]
    assert b.autotune(cache=str(tmp_path / "tune.json"))[0] == tuning  # cached
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.frag()
            b.defrag()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for r in b.restored:
            r.zero_()
        for p in b.publics:
            p.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_against_single(b, imgs, masks, ctrs, key)


@pytest.mark.parametrize("schedule", [0, 1])
def test_uneven_batch(schedule):
    """Many one-tile images around one of 12288 tiles: the tile-to-image table's
    buckets (16 tiles each here) hold up to 16 images, searched in the kernel."""
    imgs = [synth.image(8, 8 * (1 + i % 3), 1, 4, 2000 + i).cuda() for i in range(40)]
    imgs.append(synth.image(4096, 4096, 3, 4, 2040).cuda())
    imgs += [synth.image(8, 16, 1, 4, 2041 + i).cuda() for i in range(23)]
    masks = [sf.prefix_mask((1, 2, 5, 9)[i % 4]) for i in range(len(imgs))]
    ctrs = [synth.ctr0(4, 2000 + i) for i in range(len(imgs))]
    key = synth.aes_key(4)
    b = Batch(imgs, masks, key, ctrs)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.frag((1, 0, schedule), status=status)
    b.defrag((1, 0, schedule), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    _check_against_single(b, imgs, masks, ctrs, key)


def test_batch_run_rejects_unknown_schedules():
    import ctypes
    from paper_1512_02951_amd import batch as sb
    b = Batch([synth.image(16, 24, 1, 4, 0, device="cuda")], [sf.prefix_mask(2)], None, [bytes(16)])
    L = sb.lib()
    ws = ctypes.c_void_p(b.workspace.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for t in (sb.SfBatchTuning(8, 0, 2, 0), sb.SfBatchTuning(8, 0, 0, 1)):
        assert L.sf_frag_batch(ws, ctypes.byref(t), None, stream) == sf.SF_EINVAL
    assert L.sf_defrag_batch(ws, ctypes.byref(sb.SfBatchTuning(2000, 0, 1, 0)), None, stream) == sf.SF_ERANGE
    torch.cuda.synchronize()


def test_batch_plan_rejects_bad_items():
    x = torch.zeros((1, 16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SefragError):
        Batch([x, torch.zeros((1, 12, 16), dtype=torch.uint8, device="cuda")], [3, 3], None, [bytes(16)] * 2)


def test_batch_run_rejects_a_direction_without_its_image_buffers():
    # a plan whose items lack d_restored (or d_pixels) is valid for the other
    # direction only; the missing direction and the tuner (which runs both)
    # return SF_EINVAL from host validation, launching nothing
    import ctypes
    from paper_1512_02951_amd import batch as sb
    imgs = [synth.image(16, 24, 1, 4, i, device="cuda") for i in range(2)]
    b = Batch(imgs, [sf.prefix_mask(2)] * 2, None, [bytes(16)] * 2)
    L = sb.lib()
    ws = ctypes.c_void_p(b.workspace.data_ptr())
    nbytes = L.sf_batch_workspace_bytes(2)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    best, ms = sb.SfBatchTuning(), ctypes.c_float()
    b.items[1].d_restored = None
    sf.check(L.sf_batch_plan(b.items, 2, None, ws, nbytes, stream))
    assert L.sf_defrag_batch(ws, None, None, stream) == sf.SF_EINVAL
    assert L.sf_batch_autotune(ws, ctypes.byref(best), ctypes.byref(ms), stream) == sf.SF_EINVAL
    sf.check(L.sf_frag_batch(ws, None, None, stream))
    b.items[1].d_restored = b.restored[1].data_ptr()
    b.items[0].d_pixels = None
    sf.check(L.sf_batch_plan(b.items, 2, None, ws, nbytes, stream))
    assert L.sf_frag_batch(ws, None, None, stream) == sf.SF_EINVAL
    assert L.sf_batch_autotune(ws, ctypes.byref(best), ctypes.byref(ms), stream) == sf.SF_EINVAL
    sf.check(L.sf_defrag_batch(ws, None, None, stream))
    torch.cuda.synchronize()
    # the fragments written above restore both images
    for i in range(2):
        assert torch.equal(b.restored[i], imgs[i])


def test_workload4_2000_images():
    """2000 images (sides log-uniform in [256, 4096], 1 or 3 channels, k from
    {1, 2, 5, 9}, per-image nonce): every round trip exact on the GPU; 128
    sampled blocks of each of 64 images (8 per k and C) compared with the
    oracle."""
    specs = synth.batch_specs()
    key = synth.aes_key(4)
    imgs, masks, ctrs = [], [], []
    for i, (H, W, C, k) in enumerate(specs):
        imgs.append(synth.image(H, W, C, 4, i, device="cuda"))
        masks.append(sf.prefix_mask(k))
        ctrs.append(synth.ctr0(4, i))
    print("case: workload 4, %d images, %.2f G samples" % (len(imgs), sum(x.numel() for x in imgs) / 1e9), flush=True)
    b = Batch(imgs, masks, key, ctrs)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.frag(status=status)
    b.defrag(status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for i, x in enumerate(imgs):
        assert torch.equal(b.restored[i], x), "image %d round trip" % i
    rng = np.random.default_rng(44)
    chosen = []
    for k in (1, 2, 5, 9):
        for C in (1, 3):
            idx = [i for i, s in enumerate(specs) if s[3] == k and s[2] == C]
            chosen += list(rng.choice(idx, 8, replace=False))
    for i in chosen:
        H, W, C, k = specs[i]
        x = imgs[i]
        nb = C * H * W // 64
        npriv, npub = k + 1, 63 - k
        blocks = np.sort(rng.choice(nb, min(128, nb), replace=False))
        xb = x.view(C, H // 8, 8, W // 8, 8).permute(0, 1, 3, 2, 4).reshape(nb, 64)[torch.from_numpy(blocks).cuda()]
        xb = xb.cpu().numpy()
        strip = xb.reshape(-1, 8, 8).transpose(1, 0, 2).reshape(8, -1)[None]
        ref = oracle.frag(strip, masks[i])
        ref_priv = oracle.tile_unpack(ref["private"], blocks.size, npriv)
        ref_pub = oracle.tile_unpack(ref["public"], blocks.size, npub)
        prv = b.privates[i].cpu().numpy()
        for j in range(npriv):
            byte = 2 * oracle.tile_offsets(nb, npriv, blocks, j)
            ks = oracle.ctr_keystream(key, ctrs[i], byte // 16)
            k0 = ks[np.arange(byte.size), byte % 16]
            k1 = ks[np.arange(byte.size), byte % 16 + 1]
            plain = (prv[byte] ^ k0).astype(np.uint16) | ((prv[byte + 1] ^ k1).astype(np.uint16) << 8)
            assert np.array_equal(plain.view(np.int16), ref_priv[:, j])
        pidx = oracle.tile_offsets(nb, npub, np.repeat(blocks, npub), np.tile(np.arange(npub), blocks.size))
        got = b.publics[i][torch.from_numpy(pidx).cuda()].cpu().numpy().astype(np.float64).reshape(blocks.size, npub)
        nrm = np.linalg.norm(xb.astype(np.float64), axis=1)
        err = np.linalg.norm(got - ref_pub, axis=1)
        assert np.all(err[nrm == 0] == 0)
        assert (err[nrm > 0] / nrm[nrm > 0]).max() <= 1e-5
    # the static-chunk schedule on the same plan: the same fragments (checked
    # on the sampled images, bit for bit) and every round trip exact
    keep = {i: (b.publics[i].clone(), b.privates[i].clone()) for i in chosen}
    for r in b.restored:
        r.zero_()
    b.frag((2, 0, 1), status=status)
    b.defrag((2, 0, 1), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    for i, (pub, prv) in keep.items():
        assert torch.equal(pub.view(torch.int32), b.publics[i].view(torch.int32)), "image %d public (static)" % i
        assert torch.equal(prv, b.privates[i]), "image %d private (static)" % i
    for i, x in enumerate(imgs):
        assert torch.equal(b.restored[i], x), "image %d round trip (static)" % i
