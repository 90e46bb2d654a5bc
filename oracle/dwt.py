"""Plain CPU oracle of the wavelet variant -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; it shares no code with the GPU library.

Selective encryption with the LeGall 5/3 integer wavelet on 8x8 blocks
(report Sec. 6.8-6.9, Eqs. (1)-(2), Fig. 18):

* each sample is read as a signed value x - 128 (Sec. 6.9.4 treats the byte
  range as -128..127);
* one level of the 2-D transform is the 1-D lifting applied to every row, then
  to every column, of the block (Sec. 6.9.4: horizontal, then vertical); the
  outputs of a 1-D pass are stored low half then high half (Fig. 16 layout);
* the second level transforms the 4x4 low-low quarter the same way;
* the private fragment is the 2x2 second-level low-low corner (k = 4 of 64,
  Sec. 6.9.3), as int16, encrypted with AES-128-CTR as one byte stream; the
  other 60 coefficients are the public fragment, as int16.

1-D lifting on an even-length signal x (whole-sample symmetric extension,
x(-1) = x(1), x(N) = x(N - 2)):
    d(n) = x(2n+1) - floor((x(2n) + x(2n+2)) / 2)        (Eq. (1))
    s(n) = x(2n)   + floor((d(n-1) + d(n) + 2) / 4)       (Eq. (2), read as the
                                                            5/3 update step)
The inverse undoes the two steps in reverse order, so every block comes back
exactly.  Fragment layout: the tile-interleaved layout of the DCT form
(value j of block 64t + i at 64 t P + j n_t + i), P = 4 private / 60 public
values per block, public values in row-major order of their 8x8 positions.
"""
from __future__ import annotations

import numpy as np

from . import blocks_of, ctr_xor, tile_pack, tile_unpack, _planes

PRIVATE_POS = [(0, 0), (0, 1), (1, 0), (1, 1)]
PUBLIC_POS = [(r, c) for r in range(8) for c in range(8) if (r, c) not in PRIVATE_POS]


def _fdiv(a, b):
    """floor(a / b) for integer arrays (numpy // is floor division)."""
    return a // b


def lift_forward(x: np.ndarray) -> np.ndarray:
    """One 1-D 5/3 analysis along the last axis: [s | d] (low then high)."""
    x = np.asarray(x, np.int64)
    N = x.shape[-1]
    h = N // 2
    ev = x[..., 0::2]                                   # x(2n), n = 0..h-1
    od = x[..., 1::2]                                   # x(2n+1)
    ev_next = np.concatenate([ev[..., 1:], x[..., N - 2:N - 1]], axis=-1)   # x(2n+2), x(N) = x(N-2)
    d = od - _fdiv(ev + ev_next, 2)
    d_prev = np.concatenate([d[..., :1], d[..., :h - 1]], axis=-1)          # d(n-1), d(-1) = d(0)
    s = ev + _fdiv(d_prev + d + 2, 4)
    return np.concatenate([s, d], axis=-1)


def lift_inverse(y: np.ndarray) -> np.ndarray:
    """Inverse of lift_forward along the last axis."""
    y = np.asarray(y, np.int64)
    N = y.shape[-1]
    h = N // 2
    s, d = y[..., :h], y[..., h:]
    d_prev = np.concatenate([d[..., :1], d[..., :h - 1]], axis=-1)
    ev = s - _fdiv(d_prev + d + 2, 4)
    ev_next = np.concatenate([ev[..., 1:], ev[..., h - 1:h]], axis=-1)      # x(N) = x(N-2) = last even
    od = d + _fdiv(ev + ev_next, 2)
    x = np.empty(y.shape, np.int64)
    x[..., 0::2] = ev
    x[..., 1::2] = od
    return x


def level_forward(blk: np.ndarray) -> np.ndarray:
    """One 2-D level on (..., n, n): rows, then columns."""
    r = lift_forward(blk)
    return np.swapaxes(lift_forward(np.swapaxes(r, -1, -2)), -1, -2)


def level_inverse(c: np.ndarray) -> np.ndarray:
    """Inverse of level_forward: columns, then rows."""
    r = np.swapaxes(lift_inverse(np.swapaxes(c, -1, -2)), -1, -2)
    return lift_inverse(r)


def dwt_blocks(blocks: np.ndarray) -> np.ndarray:
    """(nb, 64) samples 0..255 -> (nb, 8, 8) two-level coefficients."""
    x = np.asarray(blocks, np.int64).reshape(-1, 8, 8) - 128
    c = level_forward(x)
    c[:, :4, :4] = level_forward(c[:, :4, :4])
    return c


def idwt_blocks(coef: np.ndarray) -> np.ndarray:
    """Inverse of dwt_blocks: (nb, 8, 8) -> (nb, 64) samples."""
    c = np.array(coef, np.int64)
    c[:, :4, :4] = level_inverse(c[:, :4, :4])
    return (level_inverse(c) + 128).reshape(-1, 64)


def frag(pix: np.ndarray, key: bytes | None = None, ctr0: bytes | None = None):
    """Wavelet fragmentation of planar uint8 images.  Returns dict with
    public (flat int16, tile layout, 60 per block), private (flat int16, tile
    layout, 4 per block), cipher (uint8 or None)."""
    blk = blocks_of(pix)
    c = dwt_blocks(blk)
    priv = np.stack([c[:, r, q] for r, q in PRIVATE_POS], axis=1)
    pub = np.stack([c[:, r, q] for r, q in PUBLIC_POS], axis=1)
    assert np.abs(priv).max(initial=0) < 2 ** 15 and np.abs(pub).max(initial=0) < 2 ** 15
    out = {"public": tile_pack(pub.astype(np.int16)), "private": tile_pack(priv.astype(np.int16)),
           "nb": blk.shape[0], "cipher": None}
    if key is not None:
        out["cipher"] = ctr_xor(key, ctr0 if ctr0 is not None else bytes(16), out["private"].view(np.uint8))
    return out


def defrag(shape, public: np.ndarray, private: np.ndarray | None = None, key: bytes | None = None,
           ctr0: bytes | None = None, cipher: np.ndarray | None = None) -> np.ndarray:
    """Inverse of frag: planar uint8 image of the given (C, H, W) shape."""
    C, H, W = shape
    nb = C * (H // 8) * (W // 8)
    if cipher is not None:
        private = ctr_xor(key, ctr0 if ctr0 is not None else bytes(16), np.asarray(cipher, np.uint8)).view(np.int16)
    priv = tile_unpack(np.asarray(private, np.int16), nb, 4).astype(np.int64)
    pub = tile_unpack(np.asarray(public, np.int16), nb, 60).astype(np.int64)
    c = np.zeros((nb, 8, 8), np.int64)
    for j, (r, q) in enumerate(PRIVATE_POS):
        c[:, r, q] = priv[:, j]
    for j, (r, q) in enumerate(PUBLIC_POS):
        c[:, r, q] = pub[:, j]
    x = idwt_blocks(c)
    return x.reshape(C, H // 8, W // 8, 8, 8).transpose(0, 1, 3, 2, 4).reshape(C, H, W).astype(np.uint8)


def fragment_bytes(C: int, H: int, W: int):
    """(public_bytes, private_bytes)."""
    nb = C * (H // 8) * (W // 8)
    return 2 * 60 * nb, 2 * 4 * nb


__all__ = ["lift_forward", "lift_inverse", "level_forward", "level_inverse", "dwt_blocks", "idwt_blocks", "frag",
           "defrag", "fragment_bytes", "PRIVATE_POS", "PUBLIC_POS", "_planes"]
