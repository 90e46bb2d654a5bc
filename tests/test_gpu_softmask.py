"""GPU parity of the differentiation form (soft frequency mask, hand-written
adjoint) against the FP64 oracle, through the C ABI.

Bars: public image P within 1e-5 absolute (samples in [0, 1]); every
frequency's energy E_n within a bound derived from the FP32 arithmetic (below)
and the sample sums within 1e-5 relative; loss within 1e-6 relative;
dL/dlogits within 1e-4 of the oracle normwise and every component within the
bound its own terms give; the closed form also against central differences of
itself (h = 1e-3); the tuner's loss trace and logits against the oracle's Adam.

Energy bound.  Each coefficient comes from two passes of 8-point butterflies;
every output is at most five roundings of partial sums bounded by half the
L1 norm of its inputs, so |DCT_fp32(x)_n - DCT(x)_n| <= GAMMA * ||x_blk||_1
with GAMMA = 16 u (about three times the ~5 u the passes can reach; u = 2^-24).
Squaring and summing over blocks then gives
  |E_gpu,n - E_n| <= sum_blk (2 |X_n| d + d^2) + (8 + T) u E_n,   d = GAMMA ||x_blk||_1,
the last term for the FP32 sums of non-negative terms inside a wave (a 6-level
lane tree, one square, T tiles in sequence; T <= the tiles of one image) before
they go to FP64.  Unlike a bound scaled by the DC energy, it holds each high
frequency to its own size.
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


U32 = 2.0 ** -24
GAMMA = 16 * U32


def _blocks(img):
    H, W = img.shape
    return img.reshape(H // 8, 8, W // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)


def _energy_terms(xr, gamma=GAMMA):
    """Per image and frequency: the oracle energies E (B, 64) and the bound
    on |E_gpu - E| derived in the module docstring."""
    Bm = oracle.basis()
    B, H, W = xr.shape
    T = -(-(H // 8) * (W // 8) // 64)
    E = np.empty((B, 64))
    tol = np.empty((B, 64))
    for i in range(B):
        blk = _blocks(xr[i])
        X = blk @ Bm.T
        d = gamma * np.abs(blk).sum(1)
        E[i] = (X ** 2).sum(0)
        tol[i] = 2.0 * (np.abs(X) * d[:, None]).sum(0) + (d ** 2).sum() + (8 + T) * U32 * E[i]
    return E, tol


def _assert_energies(got, xr):
    E, tol = _energy_terms(xr)
    err = np.abs(np.asarray(got, np.float64)[:, :64] - E)
    bad = np.argwhere(err > tol)
    assert bad.size == 0, "energy E_n outside its bound at (image, n) %s: err %s tol %s E %s" % (
        bad[:4].tolist(), err[tuple(bad[:4].T)], tol[tuple(bad[:4].T)], E[tuple(bad[:4].T)])


def _assert_grad_components(g, xr, l, gamma=GAMMA):
    """Every component of dL/dlogits within the error its own terms allow:
    dL/dm_n = -sum_b (a_b DCT(x - mean)_n + b_b DCT(P - mean)_n) . DCT(x)_n with
    a_b = 2 rho/(B sx sP N), b_b = -2 rho^2/(B sP^2 N); each image contributes
    (|a_b| + |b_b|) times its energy bound, the coefficients a_b, b_b and the
    mask carry 1e-5 relative, and the budget term 1e-5 of itself."""
    l = np.asarray(l, np.float64)
    B, H, W = xr.shape
    N = H * W
    gref, _, _ = oracle.softmask_grad(xr, l)
    P = oracle.softmask_public(xr, l)
    E, tolE = _energy_terms(xr, gamma)
    m = oracle.sigmoid(l)
    dsig = m * (1.0 - m)
    scale = np.zeros(64)
    for i in range(B):
        sx, sp = xr[i].std(), P[i].std()
        rho = oracle.pearson(P[i], xr[i])
        ab = abs(2.0 * rho / (B * sx * sp * N)) + abs(2.0 * rho * rho / (B * sp * sp * N))
        scale += ab * (tolE[i] + 1e-5 * E[i])
    tol = dsig * (scale + 1e-5 * 2.0 * oracle.LAMBDA * abs(m.sum() - oracle.BUDGET)) + 1e-5 * np.abs(gref)
    err = np.abs(np.asarray(g, np.float64) - gref)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, "dL/dl_n outside its bound at n = %s: err %s tol %s g %s" % (
        bad[:6].tolist(), err[bad[:6]], tol[bad[:6]], gref[bad[:6]])


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
    _assert_energies(got, xr)
    assert np.allclose(got[:, 64], sx, rtol=TOL_STATS)


@pytest.mark.parametrize("B,H,W", SHAPES[1:])
def test_closed_form_loss_and_gradient(B, H, W):
    x = _images(B, H, W)
    l = _logits()
    loss, grad = sm.closed_form(x.cuda(), _dev(l))
    gref, Lref, _ = oracle.softmask_grad(x.double().numpy(), l.astype(np.float64))
    assert abs(loss.item() - Lref) <= TOL_LOSS * abs(Lref)
    assert _normrel(grad.cpu().numpy(), gref) <= TOL_GRAD
    _assert_grad_components(grad.cpu().numpy(), x.double().numpy(), l)


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
    # this route also transforms the stored FP32 public image and G: twice the
    # transform error per block
    _assert_grad_components(l.grad.cpu().numpy(), x.cpu().double().numpy(), _logits(3), 2 * GAMMA)


def test_adjoint_kernel_for_an_arbitrary_upstream_gradient():
    B, H, W = 2, 72, 136
    x = _images(B, H, W)
    G = torch.from_numpy(np.random.default_rng(7).standard_normal((B, H, W)).astype(np.float32))
    l = _logits(5)
    g = sm.backward(x.cuda(), G.cuda(), _dev(l))
    ref = oracle.softmask_adjoint(x.double().numpy(), G.double().numpy(), l.astype(np.float64))
    assert _normrel(g.cpu().numpy(), ref) <= TOL_GRAD


def test_image_gradient_through_the_public_map():
    # x -> P is linear and symmetric, so dL/dx = P(logits) applied to dL/dP
    B, H, W = 2, 72, 136
    x = _images(B, H, W).cuda().requires_grad_(True)
    G = np.random.default_rng(11).standard_normal((B, H, W)).astype(np.float32).astype(np.float64)
    l = _logits(5)
    ld = _dev(l).requires_grad_(True)
    P = sm.SoftMaskPublic.apply(x, ld)
    (P * torch.from_numpy(G.astype(np.float32)).cuda()).sum().backward()
    gx_ref = oracle.softmask_public(G, l.astype(np.float64))
    # forward and inverse transform, each within GAMMA of the block's L1 norm
    l1 = max(np.abs(_blocks(G[i])).sum(1).max() for i in range(B))
    assert np.abs(x.grad.cpu().double().numpy() - gx_ref).max() <= 2 * GAMMA * l1
    ref = oracle.softmask_adjoint(x.detach().cpu().double().numpy(), G, l.astype(np.float64))
    assert _normrel(ld.grad.cpu().numpy(), ref) <= TOL_GRAD
    # the correlation loss differentiates with respect to P and the logits only
    with pytest.raises(ValueError):
        sm.CorrelationLoss.apply(x, P, ld, sm.LAMBDA, sm.BUDGET)


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
    _assert_energies(got, xr)
    assert np.allclose(got[:, 64], sx, rtol=TOL_STATS)
    for i in (0, 37, 63):
        Pref = oracle.softmask_public(xr[i:i + 1], l.astype(np.float64))
        assert np.abs(P[i:i + 1].cpu().double().numpy() - Pref).max() <= TOL_P
