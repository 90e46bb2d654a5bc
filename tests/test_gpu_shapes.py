"""GPU tests of the launch shapes of frag_image / defrag_image and their tuner
(sf_set_launch_shape, sf_get_launch_shape, sf_tune_image), through the C ABI.

Every shape must give the same fragments bit for bit (public values, private
bytes, exception entries, residual codes) as the default shape, whose parity
with the oracle the other GPU tests establish, and an exact round trip.
"""
import numpy as np
import pytest
import torch

import synth

sf = pytest.importorskip("paper_1512_02951_amd")

pytestmark = pytest.mark.gpu

SHAPES = [(w, r) for r in (0, 1) for w in (1, 2, 4, 6, 8)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert sf.lib().sf_init() == 0, sf.lib().sf_last_error()


def _forget(shape, mask, prec):
    for which in ("frag", "defrag"):
        sf.set_launch_shape(shape, mask, which, None, precision=prec)


def _same(a: sf.Fragments, b: sf.Fragments, label):
    assert torch.equal(a.public.view(torch.uint8), b.public.view(torch.uint8)), label
    assert torch.equal(a.private, b.private), label
    if a.residual is not None:
        assert torch.equal(a.residual, b.residual), label
    if a.exceptions is not None:
        ia, va, ca = a.exceptions.decode()
        ib, vb, cb = b.exceptions.decode()
        assert np.array_equal(ca, cb), label
        oa, ob = np.argsort(ia, kind="stable"), np.argsort(ib, kind="stable")
        assert np.array_equal(ia[oa], ib[ob]) and np.array_equal(va[oa], vb[ob]), label


CASES = [
    ("fp32", (3, 136, 264), sf.prefix_mask(5)),    # 27 tiles, the last one ragged
    ("fp32", (1, 264, 136), sf.prefix_mask(9)),    # reconstruction estimate + exceptions
    ("fp32", (1, 72, 520), 0b1011011 | (1 << 40)),  # run-time selection
    ("fp16", (1, 264, 136), sf.prefix_mask(9)),
    ("bf16", (3, 136, 264), sf.prefix_mask(2)),
]


def test_default_shapes():
    """The documented defaults: plain frag 4 waves with one tile each; plain
    defrag 2 waves with one tile each below 8 private coefficients, 4 resident
    from 8 on;
    reduced precision resident, with the largest workgroup whose LDS lets two
    share a CU (8 waves at DC + 9 AC)."""
    big = (1, 8192, 8192)
    for which in ("frag", "defrag"):
        _forget(big, sf.prefix_mask(5), "fp32")
        _forget(big, sf.prefix_mask(9), "fp32")
        _forget(big, sf.prefix_mask(9), "fp16")
        assert sf.launch_shape(big, sf.prefix_mask(5), which) == ((4, 0) if which == "frag" else (2, 0))
        assert sf.launch_shape(big, sf.prefix_mask(9), which) == (4, 0 if which == "frag" else 1)
        assert sf.launch_shape(big, sf.prefix_mask(9), which, precision="fp16") == (8, 1)


@pytest.mark.parametrize("prec,shape,mask", CASES)
def test_every_launch_shape_gives_the_default_fragments(prec, shape, mask):
    C, H, W = shape
    x = synth.image(H, W, C, 3, 7).cuda()
    key, c0 = synth.aes_key(3), synth.ctr0(3, 7)
    _forget(shape, mask, prec)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = sf.frag_image(x, mask, key, c0, precision=prec, status=status)
    torch.cuda.synchronize()
    tried = 0
    try:
        for w, r in SHAPES:
            try:
                sf.set_launch_shape(shape, mask, "frag", w, r, precision=prec)
                sf.set_launch_shape(shape, mask, "defrag", w, r, precision=prec)
            except sf.SefragError as e:  # that many waves' LDS does not fit this selection
                assert e.code == sf.SF_ENOTSUP, e
                continue
            assert sf.launch_shape(shape, mask, "frag", precision=prec) == (w, r)
            fr = sf.frag_image(x, mask, key, c0, precision=prec, status=status)
            y = sf.defrag_image(fr, key, c0, status=status)
            torch.cuda.synchronize()
            label = "%s %s mask %x shape (%d, %d)" % (prec, shape, mask, w, r)
            _same(ref, fr, label)
            assert torch.equal(x, y), label
            tried += 1
    finally:
        _forget(shape, mask, prec)
    assert tried >= 6
    assert int(status.item()) == 0


@pytest.mark.parametrize("prec,shape,mask", [("fp32", (3, 520, 264), sf.prefix_mask(5)),
                                             ("fp16", (1, 264, 520), sf.prefix_mask(9))])
def test_tuner_stores_the_fastest_shape_and_keeps_results_exact(prec, shape, mask):
    C, H, W = shape
    x = synth.image(H, W, C, 3, 11).cuda()
    key, c0 = synth.aes_key(3), synth.ctr0(3, 11)
    _forget(shape, mask, prec)
    default = (sf.launch_shape(shape, mask, "frag", precision=prec),
               sf.launch_shape(shape, mask, "defrag", precision=prec))
    assert default[0][0] >= 1 and default[1][0] >= 1
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = sf.frag_image(x, mask, key, c0, precision=prec, status=status)
    try:
        r = sf.tune_image(x, mask, key, c0, precision=prec, status=status)
        for which in ("frag", "defrag"):
            w, res = r[which]
            assert w in (1, 2, 4, 6, 8) and res in (0, 1)
            assert sf.launch_shape(shape, mask, which, precision=prec) == (w, res)
        assert r["frag_ms"] > 0 and r["defrag_ms"] > 0
        assert torch.equal(r["restored"], x)
        _same(ref, r["fragments"], "tuned")
        # the next calls use the tuned shapes and still give the same fragments
        fr = sf.frag_image(x, mask, key, c0, precision=prec, status=status)
        _same(ref, fr, "after tuning")
        assert torch.equal(sf.defrag_image(fr, key, c0, status=status), x)
    finally:
        _forget(shape, mask, prec)
    assert (sf.launch_shape(shape, mask, "frag", precision=prec),
            sf.launch_shape(shape, mask, "defrag", precision=prec)) == default
    assert int(status.item()) == 0
