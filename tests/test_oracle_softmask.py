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
