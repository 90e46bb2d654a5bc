"""Pins for the FP64 soft frequency-mask objective: special cases with closed
forms, Parseval identities, torch float64 autograd and central finite
differences."""
import numpy as np
import torch

import oracle
import synth


def _images(B=3, H=32, W=48):
    return np.stack([synth.image_plane(H, W, 5, i).numpy().astype(np.float64) / 255.0 for i in range(B)])


def test_zero_mask_gives_identity_and_loss_4_6():
    x = _images()
    logits = np.full(64, -60.0)          # sigmoid ~ 1e-26: mask ~ 0
    P = oracle.softmask_public(x, logits)
    assert np.abs(P - x).max() < 1e-12
    L = oracle.softmask_loss(x, logits)
    assert abs(L - (1.0 + 0.1 * 36.0)) < 1e-9


def test_dc_only_mask_removes_block_means():
    x = _images(B=1)
    logits = np.full(64, -60.0)
    logits[0] = 60.0
    P = oracle.softmask_public(x, logits)[0]
    H, W = x.shape[1:]
    blk = x[0].reshape(H // 8, 8, W // 8, 8)
    ref = (blk - blk.mean(axis=(1, 3), keepdims=True)).reshape(H, W)
    assert np.abs(P - ref).max() < 1e-12


def test_parseval_closed_forms_of_the_statistics():
    x = _images(B=2)
    rng = np.random.default_rng(0)
    logits = rng.standard_normal(64)
    m = oracle.sigmoid(logits)
    P = oracle.softmask_public(x, logits)
    Bm = oracle.basis()
    for i in range(x.shape[0]):
        blk = oracle._img_blocks(x[i])
        E = ((blk @ Bm.T) ** 2).sum(0)
        assert abs((P[i] * x[i]).sum() - ((1 - m) * E).sum()) < 1e-9
        assert abs((P[i] ** 2).sum() - ((1 - m) ** 2 * E).sum()) < 1e-9
        assert abs(P[i].mean() - (1 - m[0]) * x[i].mean()) < 1e-12


def _torch_loss(x, logits_t):
    Bm = torch.tensor(oracle.basis(), dtype=torch.float64)
    m = torch.sigmoid(logits_t)
    rhos = []
    for i in range(x.shape[0]):
        blk = torch.tensor(oracle._img_blocks(x[i]), dtype=torch.float64)
        P = ((blk @ Bm.T) * (1 - m)) @ Bm
        a = blk - blk.mean()
        b = P - P.mean()
        rhos.append((a * b).mean() / torch.sqrt((a * a).mean() * (b * b).mean()))
    rho = torch.stack(rhos)
    return (rho ** 2).mean() + 0.1 * (m.sum() - 6.0) ** 2


def test_gradient_matches_autograd_and_finite_differences():
    x = _images(B=2, H=16, W=24)
    logits = synth.logits_init()
    g, L, _ = oracle.softmask_grad(x, logits)
    lt = torch.tensor(logits, dtype=torch.float64, requires_grad=True)
    Lt = _torch_loss(x, lt)
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12
    assert abs(oracle.softmask_loss(x, logits) - L) < 1e-12
    ga = lt.grad.numpy()
    assert np.linalg.norm(g - ga) <= 1e-10 * np.linalg.norm(ga)
    # central differences, h = 1e-3
    h = 1e-3
    fd = np.zeros(64)
    for n in range(64):
        e = np.zeros(64)
        e[n] = h
        fd[n] = (oracle.softmask_loss(x, logits + e) - oracle.softmask_loss(x, logits - e)) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-5 * np.linalg.norm(g)


def test_adjoint_identity():
    # <IDCT a, b> = <a, DCT b> for the orthonormal basis
    rng = np.random.default_rng(1)
    a = rng.standard_normal((5, 64))
    b = rng.standard_normal((5, 64))
    Bm = oracle.basis()
    assert abs((oracle.idct_blocks(a) * b).sum() - (a * (b @ Bm.T)).sum()) < 1e-12


def test_adjoint_of_public_image_matches_finite_differences():
    # softmask_adjoint is d<G, P(l)>/dl; P is smooth in l, so central
    # differences of the functional pin it
    x = _images(B=2, H=16, W=32)
    rng = np.random.default_rng(2)
    G = rng.standard_normal(x.shape)
    logits = synth.logits_init()
    g = oracle.softmask_adjoint(x, G, logits)
    h = 1e-4
    fd = np.zeros(64)
    for n in range(64):
        e = np.zeros(64)
        e[n] = h
        fd[n] = ((G * oracle.softmask_public(x, logits + e)).sum() - (G * oracle.softmask_public(x, logits - e)).sum()) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-7 * np.linalg.norm(g)


def test_statistics_are_block_sums():
    x = _images(B=2, H=16, W=24)
    E, sx = oracle.softmask_stats(x)
    assert np.allclose(sx, x.reshape(2, -1).sum(1), rtol=1e-13)
    # Parseval: the energies add up to the sum of squares
    assert np.allclose(E.sum(1), (x ** 2).reshape(2, -1).sum(1), rtol=1e-12)
    # DC energy: each block contributes (block sum / 8)^2
    blk = x.reshape(2, 2, 8, 3, 8).sum(axis=(2, 4))
    assert np.allclose(E[:, 0], (blk ** 2).sum(axis=(1, 2)) / 64.0, rtol=1e-12)


def test_adam_descends_and_hardens_the_top_logits():
    x = _images(B=2, H=16, W=24)
    l0 = synth.logits_init()
    l1, trace = oracle.softmask_adam(x, l0, steps=30, lr=0.05)
    assert trace.shape == (30,)
    assert trace[-1] < trace[0]
    # the first step moves every logit by lr against the sign of its gradient
    g, _, _ = oracle.softmask_grad(x, l0)
    l_one, _ = oracle.softmask_adam(x, l0, steps=1, lr=0.05)
    assert np.allclose(l_one - l0, -0.05 * np.sign(g), atol=1e-6)
    mask = oracle.harden(l1, 6)
    assert bin(mask).count("1") == 6
    zz = oracle.zigzag()
    top = set(int(n) for n in np.argsort(-l1, kind="stable")[:6])
    assert {int(zz[z]) for z in range(64) if (mask >> z) & 1} == top
    # logits falling along the zigzag walk harden into DC + the first 5 AC
    ramp = np.empty(64)
    ramp[zz] = -np.arange(64.0)
    assert oracle.harden(ramp, 6) == 0b111111
    # ties go to the lower natural index: n = 0, 1, 2 sit at zigzag 0, 1, 5
    assert oracle.harden(np.zeros(64), 3) == 0b100011


def test_adam_matches_torch_optim_adam_over_many_steps():
    # The tuner's optimiser (beta1 0.9, beta2 0.999, eps 1e-8) against torch's
    # own Adam driven by the same oracle gradients: every step's logits and
    # loss agree, so the moment decays, bias corrections and step size are
    # those of the published method, not only its first step (where the
    # recurrences cancel).
    x = _images(B=2, H=16, W=24)
    l0 = synth.logits_init()
    steps, lr = 30, 0.05
    p = torch.tensor(l0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    want_trace = []
    want_logits = []
    for _ in range(steps):
        g, loss, _ = oracle.softmask_grad(x, p.detach().numpy())
        want_trace.append(loss)
        p.grad = torch.from_numpy(g)
        opt.step()
        want_logits.append(p.detach().numpy().copy())
    for t in (1, 2, 5, steps):
        lt, trace = oracle.softmask_adam(x, l0, steps=t, lr=lr)
        assert np.abs(lt - want_logits[t - 1]).max() <= 1e-12
        assert np.abs(trace - np.array(want_trace[:t])).max() <= 1e-12
    # a long run exercises the decays well past the bias-correction transient
    assert np.abs(want_logits[-1] - l0).max() > 10 * lr
