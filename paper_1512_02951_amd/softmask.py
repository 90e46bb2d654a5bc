"""Binding of the differentiation form (sf_softmask_*): argument marshalling
and buffer allocation with torch only; every step runs in the HIP library.

* :class:`SoftMaskPublic` -- ``P = SoftMaskPublic.apply(x, logits)``, the
  public image of a soft frequency mask m = sigmoid(logits) (forward kernel),
  with the hand-written adjoint kernel as its backward (gradient for the
  logits; the images are data and get none).
* :class:`CorrelationLoss` -- ``L = CorrelationLoss.apply(x, P, logits, lam,
  budget)``: mean over images of the squared correlation of P and x plus
  lam * (sum sigmoid(logits) - budget)^2; its backward writes dL/dP and the
  budget term's dL/dlogits.
* :func:`closed_form` -- loss and dL/dlogits from one statistics pass over x
  (Parseval), without forming P.
* :func:`tune` -- the Adam tuning loop on those statistics, all in one kernel,
  returning the tuned logits, the loss trace and the hardened private mask.

Images are (B, H, W) float32 CUDA tensors, H and W multiples of 8.
"""
from __future__ import annotations

import ctypes

from . import check, lib as _base_lib, _stream

LAMBDA = 0.1
BUDGET = 6.0


def _declare(L):
    P, u32, sz, i32, f32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int, ctypes.c_float
    L.sf_softmask_workspace_bytes.argtypes = [u32, u32, u32]
    L.sf_softmask_workspace_bytes.restype = sz
    L.sf_softmask_forward.argtypes = [P, u32, u32, u32, P, P, P, P, sz, P]
    L.sf_softmask_forward_noalloc.argtypes = [P, u32, u32, u32, P, P, P, P]
    L.sf_softmask_corr_stats.argtypes = [P, P, u32, u32, u32, P, P, sz, P]
    L.sf_softmask_loss.argtypes = [P, i32, P, u32, u32, u32, f32, f32, P, P, P, P, P]
    L.sf_softmask_corr_grad.argtypes = [P, P, u32, u32, u32, P, P, P, P, P, P]
    L.sf_softmask_backward.argtypes = [P, P, u32, u32, u32, P, P, P, sz, P]
    L.sf_softmask_tune.argtypes = [P, u32, u32, u32, f32, f32, u32, f32, P, P, P, u32, P]
    for n in ("sf_softmask_forward", "sf_softmask_forward_noalloc", "sf_softmask_corr_stats", "sf_softmask_loss", "sf_softmask_corr_grad",
              "sf_softmask_backward", "sf_softmask_tune"):
        getattr(L, n).restype = i32


_declared = False


def lib():
    """The shared library with the soft-mask entry points declared."""
    global _declared
    L = _base_lib()
    if not _declared:
        _declare(L)
        _declared = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_images(x):
    import torch
    if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 3 and x.is_contiguous()):
        raise ValueError("images must be a contiguous (B, H, W) float32 CUDA tensor")
    return x.shape


def _logits(logits):
    import torch
    if not (logits.is_cuda and logits.dtype == torch.float32 and logits.numel() == 64 and logits.is_contiguous()):
        raise ValueError("logits must be 64 contiguous float32 values on the GPU")
    return logits


class Workspace:
    """Device workspace of the soft-mask calls, sized for (B, H, W)."""

    def __init__(self, shape, device):
        import torch
        B, H, W = shape
        self.shape = tuple(shape)
        self.nbytes = lib().sf_softmask_workspace_bytes(B, H, W)
        self.buf = torch.empty(max(self.nbytes, 16), dtype=torch.uint8, device=device)


_ws_cache = {}


def workspace(shape, device) -> Workspace:
    key = (tuple(shape), str(device))
    ws = _ws_cache.get(key)
    if ws is None:
        ws = _ws_cache[key] = Workspace(shape, device)
    return ws


def forward(x, logits, public=True, stats=None, ws=None, stream=None):
    """(P or None, stats): P = IDCT(DCT(x) (1 - sigmoid(logits))) per block,
    stats (B, 65) float64 = E_0..E_63, sum x per image."""
    import torch
    B, H, W = _check_images(x)
    _logits(logits)
    ws = ws or workspace(x.shape, x.device)
    P = torch.empty_like(x) if public else None
    stats = stats if stats is not None else torch.empty((B, 65), dtype=torch.float64, device=x.device)
    check(lib().sf_softmask_forward(_p(x), B, H, W, _p(logits), _p(P), _p(stats), _p(ws.buf), ws.nbytes,
                                    _stream(stream)))
    return P, stats


def forward_noalloc(x, logits, public, stats, stream=None):
    """As :func:`forward` into caller-given outputs (public may be None),
    with the library's static scratch array instead of a workspace: the call
    allocates nothing.  Calls that overlap on one device race."""
    B, H, W = _check_images(x)
    _logits(logits)
    if public is not None:
        _check_images(public)
    check(lib().sf_softmask_forward_noalloc(_p(x), B, H, W, _p(logits), _p(public), _p(stats), _stream(stream)))
    return public, stats


def corr_stats(x, P, ws=None, stream=None):
    """(B, 5) float64: sum x, sum P, sum xP, sum x^2, sum P^2 per image."""
    import torch
    B, H, W = _check_images(x)
    _check_images(P)
    ws = ws or workspace(x.shape, x.device)
    st = torch.empty((B, 5), dtype=torch.float64, device=x.device)
    check(lib().sf_softmask_corr_stats(_p(x), _p(P), B, H, W, _p(st), _p(ws.buf), ws.nbytes, _stream(stream)))
    return st


def loss_from_stats(stats, logits, shape, mode, lam=LAMBDA, budget=BUDGET, gcoef=True, stream=None):
    """(loss (1,) float64, dL/dlogits or None, budget dL/dlogits, gcoef or None)."""
    import torch
    B, H, W = shape
    dev = stats.device
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(64, dtype=torch.float32, device=dev) if mode == 0 else None
    gbud = torch.empty(64, dtype=torch.float32, device=dev)
    gc = torch.empty((B, 4), dtype=torch.float32, device=dev) if gcoef else None
    check(lib().sf_softmask_loss(_p(stats), mode, _p(_logits(logits)), B, H, W, lam, budget, _p(loss), _p(grad),
                                 _p(gbud), _p(gc), _stream(stream)))
    return loss, grad, gbud, gc


def closed_form(x, logits, lam=LAMBDA, budget=BUDGET, stream=None):
    """Loss and dL/dlogits from one statistics pass over x: (loss, grad)."""
    _, stats = forward(x, logits, public=False, stream=stream)
    loss, grad, _, _ = loss_from_stats(stats, logits, x.shape, 0, lam, budget, gcoef=False, stream=stream)
    return loss, grad


def backward(x, grad_public, logits, ws=None, stream=None):
    """dL/dlogits (64 float32) for an upstream gradient dL/dP, by the adjoint kernel."""
    import torch
    B, H, W = _check_images(x)
    _check_images(grad_public)
    ws = ws or workspace(x.shape, x.device)
    g = torch.empty(64, dtype=torch.float32, device=x.device)
    check(lib().sf_softmask_backward(_p(x), _p(grad_public), B, H, W, _p(_logits(logits)), _p(g), _p(ws.buf),
                                     ws.nbytes, _stream(stream)))
    return g


def tune(x, logits, steps=200, lr=0.05, n_private=6, lam=LAMBDA, budget=BUDGET, stream=None):
    """Adam on the logits against the closed-form objective; returns
    (tuned logits, loss trace (steps,), private_mask as a Python int)."""
    import torch
    B, H, W = _check_images(x)
    l = _logits(logits).clone()
    _, stats = forward(x, l, public=False, stream=stream)
    trace = torch.empty(max(steps, 1), dtype=torch.float64, device=x.device)
    mask = torch.zeros(1, dtype=torch.int64, device=x.device)
    check(lib().sf_softmask_tune(_p(stats), B, H, W, lam, budget, steps, lr, _p(l), _p(trace), _p(mask), n_private,
                                 _stream(stream)))
    return l, trace[:steps], int(mask.item()) & ((1 << 64) - 1)


def _autograd():
    import torch

    class SoftMaskPublic(torch.autograd.Function):
        """P = IDCT(DCT(x) (1 - sigmoid(logits))); backward = adjoint kernels.

        For the logits, the hand-written adjoint kernel.  For the image, the
        map x -> P is linear with the symmetric matrix B^T diag(1 - m) B (B
        the orthonormal block basis), so its adjoint is the same map: the
        forward kernel applied to the upstream gradient."""

        @staticmethod
        def forward(ctx, x, logits):
            P, _ = forward(x, logits)
            ctx.save_for_backward(x, logits)
            return P

        @staticmethod
        def backward(ctx, gP):
            x, logits = ctx.saved_tensors
            gP = gP.contiguous()
            gx = forward(gP, logits)[0] if ctx.needs_input_grad[0] else None
            gl = backward(x, gP, logits) if ctx.needs_input_grad[1] else None
            return gx, gl

    class CorrelationLoss(torch.autograd.Function):
        """mean_b rho(P_b, x_b)^2 + lam (sum sigmoid(logits) - budget)^2."""

        @staticmethod
        def forward(ctx, x, P, logits, lam=LAMBDA, budget=BUDGET):
            if x.requires_grad:
                raise ValueError("CorrelationLoss differentiates with respect to P and the logits only; "
                                 "pass x detached (x.detach())")
            st = corr_stats(x, P)
            loss, _, gbud, gc = loss_from_stats(st, logits, x.shape, 1, lam, budget)
            ctx.save_for_backward(x, P, gc, gbud)
            return loss[0]

        @staticmethod
        def backward(ctx, gL):
            import torch
            x, P, gc, gbud = ctx.saved_tensors
            B, H, W = x.shape
            gP = torch.empty_like(P)
            gl = torch.empty(64, dtype=torch.float32, device=x.device)
            scale = gL.detach().to(torch.float64).reshape(1).contiguous()
            check(lib().sf_softmask_corr_grad(_p(x), _p(P), B, H, W, _p(gc), _p(scale), _p(gP), _p(gbud), _p(gl),
                                              _stream(None)))
            return None, gP, gl, None, None

    return SoftMaskPublic, CorrelationLoss


class _Lazy:
    def __init__(self, idx):
        self.idx = idx
        self.fn = None

    def apply(self, *args):
        if self.fn is None:
            self.fn = _autograd()[self.idx]
        return self.fn.apply(*args)


SoftMaskPublic = _Lazy(0)
CorrelationLoss = _Lazy(1)
