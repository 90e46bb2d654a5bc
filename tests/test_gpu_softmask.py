"""GPU parity of the differentiation form (soft frequency mask, hand-written
adjoint) against the FP64 oracle, through the C ABI.

Bars: public image P within 1e-5 absolute (samples in [0, 1]); per-image
statistics within 1e-5 relative; loss within 1e-6 relative; dL/dlogits
within 1e-4 of the oracle normwise (FP32 transforms and lane sums, FP64
across lanes); the closed form also against central differences of itself
(h = 1e-3); the tuner's loss trace and logits against the oracle's Adam.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import softmask as sm  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_P = 1e-5
TOL_STATS = 1e-5
TOL_LOSS = 1e-6
TOL_GRAD = 1e-4


def _images(B, H, W, workload=5):
    x = torch.stack([synth.image_plane(H, W, workload, i).to(torch.float32) / 255.0 for i in range(B)])
    return x.contiguous()


def _logits(seed=0):
    l = synth.logits_init() if seed == 0 else np.random.default_rng(seed).standard_normal(64)
    return l.astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _normrel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


SHAPES = [(1, 8, 8), (3, 40, 56), (2, 72, 136), (2, 128, 200)]


@pytest.mark.parametrize("B,H,W", SHAPES)
def test_forward_public_image_and_statistics(B, H, W):
    x = _images(B, H, W)
    l = _logits()
    P, st = sm.forward(x.cuda(), _dev(l))
    torch.cuda.synchronize()
    xr = x.double().numpy()
    lr = l.astype(np.float64)
    Pref = oracle.softmask_public(xr, lr)
    assert np.abs(P.cpu().double().numpy() - Pref).max() <= TOL_P
    E, sx = oracle.softmask_stats(xr)
    got = st.cpu().numpy()
    assert np.abs(got[:, :64] - E).max() <= TOL_STATS * E.max()
    assert np.allclose(got[:, 64], sx, rtol=TOL_STATS)


@pytest.mark.parametrize("B,H,W", SHAPES[1:])
def test_closed_form_loss_and_gradient(B, H, W):
    x = _images(B, H, W)
    l = _logits()
    loss, grad = sm.closed_form(x.cuda(), _dev(l))
    gref, Lref, _ = oracle.softmask_grad(x.double().numpy(), l.astype(np.float64))
    assert abs(loss.item() - Lref) <= TOL_LOSS * abs(Lref)
    assert _normrel(grad.cpu().numpy(), gref) <= TOL_GRAD


@pytest.mark.parametrize("B,H,W", SHAPES[1:])
def test_autograd_route_matches_oracle(B, H, W):
    x = _images(B, H, W).cuda()
    l = _dev(_logits(3)).requires_grad_(True)
    P = sm.SoftMaskPublic.apply(x, l)
    L = sm.CorrelationLoss.apply(x, P, l, sm.LAMBDA, sm.BUDGET)
    L.backward()
    gref, Lref, _ = oracle.softmask_grad(x.cpu().double().numpy(), _logits(3).astype(np.float64))
    assert abs(L.item() - Lref) <= TOL_LOSS * abs(Lref)
    assert _normrel(l.grad.cpu().numpy(), gref) <= TOL_GRAD


def test_adjoint_kernel_for_an_arbitrary_upstream_gradient():
    B, H, W = 2, 72, 136
    x = _images(B, H, W)
    G = torch.from_numpy(np.random.default_rng(7).standard_normal((B, H, W)).astype(np.float32))
    l = _logits(5)
    g = sm.backward(x.cuda(), G.cuda(), _dev(l))
    ref = oracle.softmask_adjoint(x.double().numpy(), G.double().numpy(), l.astype(np.float64))
    assert _normrel(g.cpu().numpy(), ref) <= TOL_GRAD


def test_closed_form_against_its_finite_differences():
    B, H, W = 2, 72, 136
    x = _images(B, H, W).cuda()
    l = _logits()
    _, stats = sm.forward(x, _dev(l), public=False)
    _, grad, _, _ = sm.loss_from_stats(stats, _dev(l), x.shape, 0, gcoef=False)
    g = grad.cpu().numpy().astype(np.float64)
    h = 1e-3
    fd = np.zeros(64)
    for n in range(64):
        lp, lm = l.copy(), l.copy()
        lp[n] += h
        lm[n] -= h
        Lp = sm.loss_from_stats(stats, _dev(lp), x.shape, 0, gcoef=False)[0].item()
        Lm = sm.loss_from_stats(stats, _dev(lm), x.shape, 0, gcoef=False)[0].item()
        fd[n] = (Lp - Lm) / (float(lp[n]) - float(lm[n]))
    assert _normrel(g, fd) <= 1e-3


def test_budget_term_alone():
    # a black image: every correlation term is 0/0 guarded to 0, only the
    # budget penalty is left, in closed form
    x = torch.zeros((1, 16, 16), dtype=torch.float32, device="cuda")
    l = _logits()
    loss, grad = sm.closed_form(x, _dev(l))
    m = oracle.sigmoid(l.astype(np.float64))
    over = m.sum() - 6.0
    # lam travels as a float32 (0.1 to 1.5e-8 relative)
    assert abs(loss.item() - 0.1 * over * over) <= 1e-7 * 0.1 * over * over
    assert _normrel(grad.cpu().numpy(), m * (1 - m) * 0.2 * over) <= 1e-6


def test_tuner_matches_oracle_adam_and_hardens_the_mask():
    B, H, W = 2, 72, 136
    x = _images(B, H, W)
    l0 = _logits()
    steps, lr = 25, 0.05
    lt, trace, mask = sm.tune(x.cuda(), _dev(l0), steps=steps, lr=lr, n_private=6)
    lref, tref = oracle.softmask_adam(x.double().numpy(), l0.astype(np.float64), steps, lr)
    tr = trace.cpu().numpy()
    assert np.all(np.abs(tr - tref) <= 1e-5 * np.abs(tref))
    assert np.abs(lt.cpu().numpy() - lref).max() <= 1e-4
    assert mask == oracle.harden(lt.cpu().numpy(), 6)
    assert bin(mask).count("1") == 6
    # the hardened mask is a valid selection for the plain path
    img = synth.image(H, W, 1, 5, 0, device="cuda")
    fr = sf.frag_image(img, mask, key=bytes(16), ctr0=bytes(16))
    out = sf.defrag_image(fr, key=bytes(16), ctr0=bytes(16))
    torch.cuda.synchronize()
    assert torch.equal(out, img)


@pytest.mark.parametrize("B", [94, 100])
def test_tuner_at_and_beyond_the_lds_statistics_limit(B):
    # the tuner stages B x 65 statistics in LDS up to 94 images (48 880 of
    # 49 152 bytes); at 100 every step reads them from global memory
    H, W = 8, 16
    x = _images(B, H, W)
    l0 = _logits(3)
    steps, lr = 10, 0.05
    lt, trace, mask = sm.tune(x.cuda(), _dev(l0), steps=steps, lr=lr, n_private=6)
    lref, tref = oracle.softmask_adam(x.double().numpy(), l0.astype(np.float64), steps, lr)
    tr = trace.cpu().numpy()
    assert np.all(np.abs(tr - tref) <= 1e-5 * np.abs(tref))
    assert np.abs(lt.cpu().numpy() - lref).max() <= 1e-4
    assert mask == oracle.harden(lt.cpu().numpy(), 6)


def test_shape_errors():
    x = torch.zeros((1, 12, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(sf.SefragError) as e:
        sm.forward(x, _dev(_logits()))
    assert e.value.code == sf.SF_ESHAPE


def test_full_size_64_images_1024_squared():
    B, H, W = 64, 1024, 1024
    x = synth.softmask_images(B, H, W, device="cuda")
    l = _logits()
    ld = _dev(l)
    P, st = sm.forward(x, ld)
    loss, grad = sm.closed_form(x, ld)
    lg = ld.clone().requires_grad_(True)
    La = sm.CorrelationLoss.apply(x, sm.SoftMaskPublic.apply(x, lg), lg, sm.LAMBDA, sm.BUDGET)
    La.backward()
    torch.cuda.synchronize()
    xr = x.cpu().double().numpy()
    gref, Lref, _ = oracle.softmask_grad(xr, l.astype(np.float64))
    assert abs(loss.item() - Lref) <= TOL_LOSS * abs(Lref)
    assert abs(La.item() - Lref) <= TOL_LOSS * abs(Lref)
    assert _normrel(grad.cpu().numpy(), gref) <= TOL_GRAD
    assert _normrel(lg.grad.cpu().numpy(), gref) <= TOL_GRAD
    E, sx = oracle.softmask_stats(xr)
    got = st.cpu().numpy()
    assert np.abs(got[:, :64] - E).max() <= TOL_STATS * E.max()
    assert np.allclose(got[:, 64], sx, rtol=TOL_STATS)
    for i in (0, 37, 63):
        Pref = oracle.softmask_public(xr[i:i + 1], l.astype(np.float64))
        assert np.abs(P[i:i + 1].cpu().double().numpy() - Pref).max() <= TOL_P
