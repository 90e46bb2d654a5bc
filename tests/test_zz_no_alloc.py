"""GPU test of the allocation-free soft-mask forward (sf_softmask_forward_noalloc)
through the C ABI: its public image and statistics must equal, bit for bit,
those of sf_softmask_forward with a caller workspace on the same inputs (the
two run the same kernels on the same launch geometry).  Two calls in a row,
the second on a smaller batch, so a stale partial sum left in the shared
static array by the first call would show; then a batch too large for the
array is refused on the host before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

import synth

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import softmask as sm  # noqa: E402

pytestmark = pytest.mark.gpu


def _images(B, H, W, first=0):
    x = torch.stack([synth.image_plane(H, W, 5, first + i).to(torch.float32) / 255.0 for i in range(B)])
    return x.contiguous().cuda()


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _with_workspace(x, logits):
    L = sm.lib()
    B, H, W = x.shape
    nbytes = L.sf_softmask_workspace_bytes(B, H, W)
    ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=x.device)
    P = torch.empty_like(x)
    st = torch.empty((B, 65), dtype=torch.float64, device=x.device)
    rc = L.sf_softmask_forward(_p(x), B, H, W, _p(logits), _p(P), _p(st), _p(ws), nbytes, None)
    assert rc == sf.SF_OK, L.sf_last_error()
    return P, st


def _noalloc(x, logits, public=True):
    L = sm.lib()
    B, H, W = x.shape
    P = torch.full_like(x, float("nan")) if public else None
    st = torch.full((B, 65), float("nan"), dtype=torch.float64, device=x.device)
    rc = L.sf_softmask_forward_noalloc(_p(x), B, H, W, _p(logits), _p(P), _p(st), None)
    assert rc == sf.SF_OK, L.sf_last_error()
    return P, st


def test_noalloc_forward_equals_workspace_forward_on_two_calls():
    logits = torch.from_numpy(np.random.default_rng(3).standard_normal(64).astype(np.float32)).cuda()
    # first call: 24 images of 256 x 200 (ragged last tile), then 5 images of
    # 72 x 136: fewer workgroup partials than the first call left behind
    for B, H, W, first in ((24, 256, 200, 0), (5, 72, 136, 40)):
        x = _images(B, H, W, first)
        P_ref, st_ref = _with_workspace(x, logits)
        P, st = _noalloc(x, logits)
        torch.cuda.synchronize()
        print("noalloc forward B=%d H=%d W=%d" % (B, H, W), flush=True)
        assert torch.equal(P, P_ref)
        assert torch.equal(st, st_ref)
    # statistics only (no public image) after the others
    _, st = _noalloc(x, logits, public=False)
    torch.cuda.synchronize()
    assert torch.equal(st, st_ref)


def test_noalloc_forward_refuses_a_batch_beyond_the_scratch_array():
    L = sm.lib()
    B, H, W = 4096, 8, 8
    assert L.sf_softmask_workspace_bytes(B, H, W) > (1 << 20)
    x = torch.zeros((B, H, W), dtype=torch.float32, device="cuda")
    logits = torch.zeros(64, dtype=torch.float32, device="cuda")
    st = torch.zeros((B, 65), dtype=torch.float64, device="cuda")
    rc = L.sf_softmask_forward_noalloc(_p(x), B, H, W, _p(logits), None, _p(st), None)
    assert rc == sf.SF_ERANGE
    assert b"scratch" in L.sf_last_error()
    torch.cuda.synchronize()
    assert not st.any()  # nothing was launched
