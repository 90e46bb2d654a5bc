"""Plain CPU oracle of the pixel-domain fragment formats -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; it shares no code with the GPU library.

The report's own storage formats (Sec. 6.3.1-6.3.2, Sec. 6.4.3, Figs. 6-8,
Table 5), numpy integer arithmetic plus hashlib's SHA-512:

* private part: the integer private coefficients (rule Q2 of the DCT form,
  ``oracle.q2_blocks``) in zigzag order, each stored in 11 bits (Sec. 6.4.3):
  DC unsigned (0..2040), AC as a sign bit above a 10-bit magnitude.  The 11-bit
  fields of the blocks of a 64-block tile follow each other in one little-endian
  bit stream (field j of block i of the tile at bit 11 (i P + j), P fields per
  block); a full tile takes 88 P bytes and starts on a 16-byte boundary
  (stride 16 ceil(88 P / 16)), the last tile takes ceil(11 P n_t / 8) bytes.
  The whole private byte string is AES-128-CTR encrypted as in the DCT form
  (the counter of tile t starts at block t * stride / 16).
* public part: one byte per sample, image layout.  The report stores the
  inverse DCT of the remaining coefficients (private ones set to zero) as
  bytes.  Here that image is represented by P = (x - R) mod 256, where
  R = floor((sum_j q_j Bi[n_j][p] + 2^15) / 2^16) (round half up),
  Bi = rhe(2^16 B), is the integer inverse of the private integers: since x = IDCT(private part) +
  IDCT(rest) exactly, P differs from the inverse transform of the rest only by
  how far R is from IDCT(private part) (a bound is checked in the tests), and
  (R + P) mod 256 gives x back exactly.
* strong level (Sec. 6.3.2, Fig. 8): the 64 public bytes of a block are
  XORed with the SHA-512 digest (FIPS 180-4) of the block's private integers
  as stored, int16 little-endian in zigzag order; digest byte p masks sample
  p = 8y + x.
* 8-bit storage (Sec. 6.4.3, Table 5, lossy): AC fields of a sign bit above a
  7-bit magnitude, clamped to 127; DC keeps 11 bits.  The public part is made
  from the exact integers (as the report's public image does not depend on how
  the private part is stored), so defragmentation restores x exactly wherever
  no private AC was clamped and loses only what the clamping removed.
  ``ac_bits`` = 10 (11-bit fields, the default) or 7 (8-bit fields).
"""
from __future__ import annotations

import hashlib

import numpy as np

from . import basis, blocks_of, ctr_xor, popcount, q2_blocks, zigzag, _planes

FIELD_BITS = 11
INV_SHIFT = 16


def inv_table() -> np.ndarray:
    """Bi[n][p] = round_half_even(2^16 B[n][p]) as int64 (64 x 64)."""
    s = basis() * (1 << INV_SHIFT)
    # every entry is far from a rounding tie, so FP64 decides it exactly
    assert np.abs(s - np.floor(s) - 0.5).min() > 1e-6
    return np.rint(s).astype(np.int64)


def rhe_shift(a: np.ndarray, s: int) -> np.ndarray:
    """round_half_even(a / 2^s) for int64 arrays."""
    a = np.asarray(a, np.int64)
    fl = a >> s                                  # floor
    rem = a - (fl << s)                          # 0 .. 2^s - 1
    half = 1 << (s - 1)
    up = (rem > half) | ((rem == half) & ((fl & 1) == 1))
    return fl + up.astype(np.int64)


def private_positions(mask: int):
    """(zigzag positions, natural indices) of the private coefficients."""
    zz = zigzag()
    zpos = [z for z in range(64) if (mask >> z) & 1]
    return zpos, [int(zz[z]) for z in zpos]


def private_ints(pix: np.ndarray, mask: int) -> np.ndarray:
    """(nb, P) int64 private integers in zigzag order (rule Q2)."""
    _, nat = private_positions(mask)
    return q2_blocks(pix, nat).astype(np.int64)


def recon_private(q: np.ndarray, mask: int) -> np.ndarray:
    """R: (nb, 64) integer inverse of the private integers."""
    _, nat = private_positions(mask)
    Bi = inv_table()
    acc = np.asarray(q, np.int64) @ Bi[nat]       # (nb, 64), exact in int64
    return (acc + (1 << (INV_SHIFT - 1))) >> INV_SHIFT   # round half up


def strong_keystream(q: np.ndarray) -> np.ndarray:
    """(nb, 64) uint8: SHA-512 of each block's private integers (int16 LE)."""
    q = np.asarray(q, np.int64)
    assert np.abs(q).max(initial=0) < 2 ** 15
    msgs = q.astype("<i2")
    out = np.empty((q.shape[0], 64), np.uint8)
    for b in range(q.shape[0]):
        out[b] = np.frombuffer(hashlib.sha512(msgs[b].tobytes()).digest(), np.uint8)
    return out


def field_widths(mask: int, ac_bits: int = 10):
    """Bits of each private field in zigzag order: 11 for DC, ac_bits + 1 for AC."""
    zpos, _ = private_positions(mask)
    return [FIELD_BITS if z == 0 else ac_bits + 1 for z in zpos]


def record_bits(mask: int, ac_bits: int = 10) -> int:
    return sum(field_widths(mask, ac_bits))


def stored_ints(q: np.ndarray, mask: int, ac_bits: int = 10) -> np.ndarray:
    """The private integers as the fields hold them: AC magnitudes clamped to
    2^ac_bits - 1 (no clamping ever happens at 10 bits: |AC| <= 1020)."""
    zpos, _ = private_positions(mask)
    q = np.array(q, np.int64)
    lim = (1 << ac_bits) - 1
    for j, z in enumerate(zpos):
        if z != 0:
            q[:, j] = np.clip(q[:, j], -lim, lim)
    return q


def _fields(q: np.ndarray, mask: int, ac_bits: int = 10) -> np.ndarray:
    zpos, _ = private_positions(mask)
    q = stored_ints(q, mask, ac_bits)
    f = np.empty(q.shape, np.int64)
    for j, z in enumerate(zpos):
        if z == 0:
            assert q[:, j].min(initial=0) >= 0 and q[:, j].max(initial=0) < 2 ** FIELD_BITS
            f[:, j] = q[:, j]
        else:
            f[:, j] = np.abs(q[:, j]) | ((q[:, j] < 0).astype(np.int64) << ac_bits)
    return f


def _unfields(f: np.ndarray, mask: int, ac_bits: int = 10) -> np.ndarray:
    zpos, _ = private_positions(mask)
    q = np.empty(f.shape, np.int64)
    for j, z in enumerate(zpos):
        if z == 0:
            q[:, j] = f[:, j]
        else:
            mag = f[:, j] & ((1 << ac_bits) - 1)
            q[:, j] = np.where((f[:, j] >> ac_bits) & 1, -mag, mag)
    return q


def tile_stride(P: int, rec_bits: int | None = None) -> int:
    """Bytes per full tile: 64 records of rec_bits (11 P by default), rounded up to 16."""
    rb = FIELD_BITS * P if rec_bits is None else rec_bits
    return 16 * ((8 * rb + 15) // 16)


def private_bytes(nb: int, P: int, rec_bits: int | None = None) -> int:
    if nb == 0:
        return 0
    rb = FIELD_BITS * P if rec_bits is None else rec_bits
    nt_last = nb - 64 * ((nb - 1) // 64)
    return ((nb - 1) // 64) * tile_stride(P, rb) + (rb * nt_last + 7) // 8


def pack11(q: np.ndarray, mask: int, ac_bits: int = 10) -> np.ndarray:
    """(nb, P) private integers -> packed private bytes (tile streams); the
    fields of a record follow each other, a tile's records likewise."""
    f = _fields(q, mask, ac_bits)
    widths = field_widths(mask, ac_bits)
    nb, P = f.shape
    rb = sum(widths)
    out = np.zeros(private_bytes(nb, P, rb), np.uint8)
    st = tile_stride(P, rb)
    for t0 in range(0, nb, 64):
        ft = f[t0:t0 + 64]
        bits = np.concatenate([((ft[:, j:j + 1] >> np.arange(w)) & 1) for j, w in enumerate(widths)], axis=1)
        by = np.packbits(bits.astype(np.uint8).reshape(-1), bitorder="little")
        base = (t0 // 64) * st
        out[base:base + by.size] = by
    return out


def unpack11(data: np.ndarray, nb: int, mask: int, ac_bits: int = 10) -> np.ndarray:
    """Inverse of pack11 (returns the stored integers)."""
    P = popcount(mask)
    widths = field_widths(mask, ac_bits)
    rb = sum(widths)
    data = np.asarray(data, np.uint8)
    st = tile_stride(P, rb)
    f = np.zeros((nb, P), np.int64)
    offs = np.concatenate([[0], np.cumsum(widths)])
    for t0 in range(0, nb, 64):
        nt = min(64, nb - t0)
        nbits = rb * nt
        base = (t0 // 64) * st
        bits = np.unpackbits(data[base:base + (nbits + 7) // 8], bitorder="little")[:nbits].reshape(nt, rb)
        for j, w in enumerate(widths):
            f[t0:t0 + nt, j] = (bits[:, offs[j]:offs[j] + w].astype(np.int64) << np.arange(w)).sum(-1)
    return _unfields(f, mask, ac_bits)


def _unblocks(v: np.ndarray, shape) -> np.ndarray:
    C, H, W = shape
    return v.reshape(C, H // 8, W // 8, 8, 8).transpose(0, 1, 3, 2, 4).reshape(C, H, W)


def frag(pix: np.ndarray, mask: int, strong: bool = False, key: bytes | None = None, ctr0: bytes | None = None,
         ac_bits: int = 10):
    """Returns dict: public (C, H, W) uint8, private (packed plain bytes),
    cipher (bytes or None), q (nb, P) private integers (exact, before any
    clamping of the stored fields)."""
    pix = _planes(pix)
    blk = blocks_of(pix).astype(np.int64)
    q = private_ints(pix, mask)
    R = recon_private(q, mask)
    pub = ((blk - R) & 0xFF).astype(np.uint8)
    if strong:
        pub ^= strong_keystream(stored_ints(q, mask, ac_bits))
    plain = pack11(q, mask, ac_bits)
    out = {"public": _unblocks(pub, pix.shape), "private": plain, "cipher": None, "q": q}
    if key is not None:
        out["cipher"] = ctr_xor(key, ctr0 if ctr0 is not None else bytes(16), plain)
    return out


def defrag(shape, mask: int, public: np.ndarray, private: np.ndarray | None = None, strong: bool = False,
           key: bytes | None = None, ctr0: bytes | None = None, cipher: np.ndarray | None = None,
           ac_bits: int = 10) -> np.ndarray:
    C, H, W = shape
    nb = C * (H // 8) * (W // 8)
    if cipher is not None:
        private = ctr_xor(key, ctr0 if ctr0 is not None else bytes(16), np.asarray(cipher, np.uint8))
    q = unpack11(private, nb, mask, ac_bits)
    pub = blocks_of(np.asarray(public, np.uint8).reshape(C, H, W)).copy()
    if strong:
        pub ^= strong_keystream(q)
    x = (recon_private(q, mask) + pub.astype(np.int64)) & 0xFF
    return _unblocks(x.astype(np.uint8), shape)


def fragment_bytes(C: int, H: int, W: int, mask: int, ac_bits: int = 10):
    """(public_bytes, private_bytes)."""
    nb = C * (H // 8) * (W // 8)
    return C * H * W, private_bytes(nb, popcount(mask), record_bits(mask, ac_bits))


__all__ = ["inv_table", "rhe_shift", "private_positions", "private_ints", "recon_private", "strong_keystream",
           "field_widths", "record_bits", "stored_ints", "tile_stride", "private_bytes", "pack11", "unpack11", "frag",
           "defrag", "fragment_bytes"]
