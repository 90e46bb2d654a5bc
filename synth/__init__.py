"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the fragmentation method: it only makes
images, keys and nonces.  The report measures on natural test images that are
not available; these synthetic images stand in for them (smooth content plus
sensor-like noise, 8 bits per sample, planar channels).

Image recipe (one plane of H x W samples, image ``i``, channel ``c`` of
workload ``w``):

  v(y, x) = 128 + sum_{s=1..8} A_s sin(2 pi (x cos th_s + y sin th_s) / T_s + ph_s) + 2 n(y, x)
  pixel   = clamp(round_half_even(v), 0, 255)

* A_s ~ U[5, 30], T_s ~ U[4, 128] px, th_s, ph_s ~ U[0, 2 pi), drawn in that
  order per sinusoid from numpy PCG64 seeded by SeedSequence([151202951, w, i, c]).
* n(y, x) ~ N(0, 1) (variance of 2 n is 4) by Box-Muller from two counter-based
  uniforms u = (h + 0.5) / 2^32, h = lowbias32(lowbias32(j ^ ka) ^ kb), where j
  = y*W + x and (ka, kb) are per-stream keys drawn from the same generator.
  lowbias32 is C. Wellons' 32-bit integer mixer
  (x ^= x>>16; x *= 0x7feb352d; x ^= x>>15; x *= 0x846ca68b; x ^= x>>16).
* The sinusoid is evaluated as sin(a_x + b_y) = sin(b_y) cos(a_x) + cos(b_y) sin(a_x)
  (outer products), which is the definition used here.

Everything is torch float64/int64 arithmetic, so the same function runs on the
CPU or on the GPU (only to produce inputs faster; transcendental rounding may
differ in the last ulp between devices, so tests always hand the *same* tensor
to both sides).

Workloads
---------
1: one 512x512 grayscale image, private = DC + 2 AC (k = 2)
2: one 4096x4096 RGB planar image, k = 5 (the throughput workload)
3: 16 grayscale 8192x8192 images, k = 9 (reduced-precision form)
4: 2000 images, width/height log-uniform in [256, 4096] rounded to x8,
   1 or 3 channels (p = 1/2), k from {1, 2, 5, 9} (batched form)
5: 64 grayscale 1024x1024 images as float32 pixel/255 (soft-mask form)
The wavelet form runs on workload 2's images and key.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

SEED = 151202951


def _rng(*words) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, *words])))


def sinusoid_params(workload: int, image: int, channel: int):
    """(8, 4) float64 [A, T, theta, phi] and two 32-bit noise keys per stream."""
    r = _rng(workload, image, channel)
    p = np.zeros((8, 4), np.float64)
    for s in range(8):
        p[s, 0] = r.uniform(5.0, 30.0)
        p[s, 1] = r.uniform(4.0, 128.0)
        p[s, 2] = r.uniform(0.0, 2 * math.pi)
        p[s, 3] = r.uniform(0.0, 2 * math.pi)
    keys = r.integers(0, 1 << 32, size=4, dtype=np.uint64).astype(np.int64)
    return p, keys


_M32 = (1 << 32) - 1


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2^32 for 0 <= x < 2^32 without int64 overflow."""
    lo = x & 0xFFFF
    hi = x >> 16
    return ((((hi * c) & 0xFFFF) << 16) + lo * c) & _M32


def lowbias32(x: torch.Tensor) -> torch.Tensor:
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def _uniform(j: torch.Tensor, ka: int, kb: int) -> torch.Tensor:
    h = lowbias32(lowbias32(j ^ ka) ^ kb)
    return (h.to(torch.float64) + 0.5) / 4294967296.0


def image_plane(H: int, W: int, workload: int, image: int = 0, channel: int = 0, device="cpu") -> torch.Tensor:
    """One uint8 plane (H, W) of the recipe above."""
    p, keys = sinusoid_params(workload, image, channel)
    dev = torch.device(device)
    xs = torch.arange(W, dtype=torch.float64, device=dev)
    ys = torch.arange(H, dtype=torch.float64, device=dev)
    v = torch.full((H, W), 128.0, dtype=torch.float64, device=dev)
    for s in range(8):
        A, T, th, ph = (float(t) for t in p[s])
        a = 2 * math.pi * xs * math.cos(th) / T
        b = 2 * math.pi * ys * math.sin(th) / T + ph
        v += A * (torch.outer(torch.sin(b), torch.cos(a)) + torch.outer(torch.cos(b), torch.sin(a)))
    j = torch.arange(H * W, dtype=torch.int64, device=dev).view(H, W)
    u1 = _uniform(j, int(keys[0]), int(keys[1]))
    u2 = _uniform(j, int(keys[2]), int(keys[3]))
    n = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2 * math.pi * u2)
    del j, u1, u2
    v += 2.0 * n
    return torch.clamp(torch.round(v), 0, 255).to(torch.uint8)


def image(H: int, W: int, C: int, workload: int, image_index: int = 0, device="cpu", out: torch.Tensor | None = None) -> torch.Tensor:
    """Planar uint8 image (C, H, W)."""
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.uint8, device=device)
    for c in range(C):
        out[c] = image_plane(H, W, workload, image_index, c, device=device)
    return out


def aes_key(workload: int) -> bytes:
    return _rng(workload, 0xAE5).integers(0, 256, size=16, dtype=np.uint8).tobytes()


def ctr0(workload: int, image_index: int = 0) -> bytes:
    """8-byte per-image nonce followed by a zero 64-bit block counter."""
    return _rng(workload, image_index, 0x4E).integers(0, 256, size=8, dtype=np.uint8).tobytes() + bytes(8)


def prefix_mask(k: int) -> int:
    return (1 << (k + 1)) - 1


@dataclass(frozen=True)
class Workload:
    index: int
    name: str
    images: int
    H: int
    W: int
    C: int
    k: int


WORKLOADS = {
    1: Workload(1, "512x512 gray, k=2", 1, 512, 512, 1, 2),
    2: Workload(2, "4096x4096 RGB planar, k=5", 1, 4096, 4096, 3, 5),
    3: Workload(3, "16 x 8192x8192 gray, k=9", 16, 8192, 8192, 1, 9),
    5: Workload(5, "64 x 1024x1024 gray float32 in [0,1]", 64, 1024, 1024, 1, 5),
}


def batch_specs(n: int = 2000, workload: int = 4):
    """Per-image (H, W, C, k) of the batched workload: sides log-uniform in
    [256, 4096] rounded to multiples of 8, C = 3 with probability 1/2,
    k uniform over {1, 2, 5, 9}."""
    r = _rng(workload)
    specs = []
    lo, hi = math.log(256.0), math.log(4096.0)
    for _ in range(n):
        w = int(8 * round(math.exp(r.uniform(lo, hi)) / 8))
        h = int(8 * round(math.exp(r.uniform(lo, hi)) / 8))
        c = 3 if r.uniform() < 0.5 else 1
        k = int((1, 2, 5, 9)[r.integers(0, 4)])
        specs.append((h, w, c, k))
    return specs


def softmask_images(B: int = 64, H: int = 1024, W: int = 1024, device="cpu") -> torch.Tensor:
    """(B, H, W) float32 = generator / 255 (workload 5)."""
    out = torch.empty((B, H, W), dtype=torch.float32, device=device)
    for i in range(B):
        out[i] = image_plane(H, W, 5, i, 0, device=device).to(torch.float32) / 255.0
    return out


def logits_init(workload: int = 5) -> np.ndarray:
    """64 initial logits ~ N(0, 1)."""
    return _rng(workload, 0x106).standard_normal(64)
