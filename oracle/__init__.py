"""Plain CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it and it
imports nothing from the GPU library; the two share no code.  The only module
both sides use is ``synth`` (seeded synthetic inputs, no method arithmetic).

Contents
--------
* ``oracle.c`` (built to ``liboracle.so`` with gcc/OpenMP): FP64 direct-sum
  8x8 DCT/IDCT, JPEG zigzag, integer private quantiser, textbook AES-128 and
  CTR mode, and the whole frag/defrag pipeline of the report's first level of
  protection (Sec. 6.3.1, Fig. 6; Sec. 6.4.3).
* The soft frequency-mask objective in FP64 (numpy): public image
  P = IDCT(DCT(x) * (1 - sigmoid(l))) following the zero-padded public image of
  Sec. 6.3.1/Fig. 7, Pearson correlation of Sec. 6.6.2, loss and gradient.
* ``oracle.dwt``: the LeGall 5/3 wavelet variant (Sec. 6.8-6.9, Eqs. (1)-(2)).
* ``oracle.pixel``: the report's storage formats (11-bit and 8-bit private
  fields, public bytes in the pixel domain) and the SHA-512 strong level
  (Sec. 6.3.2, 6.4.3).
* ``oracle.stats``: the security statistics of Sec. 6.6 and 6.10.

Every function is pinned in ``tests/test_oracle_*.py`` against something other
than itself (closed forms, scipy, published AES/CTR and SHA-512 vectors,
openssl, mpmath, brute force, finite differences, values the report prints).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        lib.orc_basis.argtypes = [P]
        lib.orc_zigzag.argtypes = [P]
        lib.orc_q2_table.argtypes = [P]
        lib.orc_tile_offset.argtypes = [i64, i64, i64, i64]
        lib.orc_tile_offset.restype = i64
        lib.orc_dct_blocks.argtypes = [P, i32, i32, i32, P]
        lib.orc_idct_blocks.argtypes = [P, i64, P]
        lib.orc_q2_blocks.argtypes = [P, i32, i32, i32, P, i32, P]
        lib.orc_aes_sbox.argtypes = [P]
        lib.orc_aes_expand.argtypes = [P, P]
        lib.orc_aes128_encrypt.argtypes = [P, P, P]
        lib.orc_ctr_xor.argtypes = [P, P, u64, P, P, i64]
        lib.orc_ctr_keystream.argtypes = [P, P, P, i64, P]
        lib.orc_frag.argtypes = [P, i32, i32, i32, u64, P, P, P, P, P, P, P, i64, P]
        lib.orc_frag.restype = i64
        lib.orc_defrag.argtypes = [i32, i32, i32, u64, P, P, P, P, P, P, P, i64, P]
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_get_threads.restype = i32
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    _lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_lib().orc_get_threads())


# ---------------------------------------------------------------- transform
def basis() -> np.ndarray:
    """64x64 orthonormal 8x8 DCT-II basis B[n, p], n = 8u+v, p = 8y+x."""
    B = np.zeros((64, 64), np.float64)
    _lib().orc_basis(_ptr(B))
    return B


def zigzag() -> np.ndarray:
    """zz[z] = natural index 8u+v of zigzag position z (JPEG order)."""
    zz = np.zeros(64, np.int32)
    _lib().orc_zigzag(_ptr(zz))
    return zz


def q2_table() -> np.ndarray:
    """round_half_even(2^20 * B) as int32, 64x64."""
    t = np.zeros((64, 64), np.int32)
    _lib().orc_q2_table(_ptr(t))
    return t


def _planes(pix: np.ndarray) -> np.ndarray:
    pix = np.ascontiguousarray(pix, dtype=np.uint8)
    if pix.ndim == 2:
        pix = pix[None]
    assert pix.ndim == 3 and pix.shape[1] % 8 == 0 and pix.shape[2] % 8 == 0
    return pix


def dct_blocks(pix: np.ndarray) -> np.ndarray:
    """FP64 DCT of every 8x8 block; returns (nb, 64) in natural order."""
    pix = _planes(pix)
    C, H, W = pix.shape
    nb = C * (H // 8) * (W // 8)
    out = np.zeros((nb, 64), np.float64)
    _lib().orc_dct_blocks(_ptr(pix), C, H, W, _ptr(out))
    return out


def idct_blocks(coef: np.ndarray) -> np.ndarray:
    """FP64 inverse DCT of (nb, 64) natural-order coefficients -> (nb, 64) pixels p = 8y+x."""
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nb = coef.shape[0]
    out = np.zeros((nb, 64), np.float64)
    _lib().orc_idct_blocks(_ptr(coef), nb, _ptr(out))
    return out


def q2_blocks(pix: np.ndarray, nat) -> np.ndarray:
    """Integer private quantiser for the natural indices ``nat``: (nb, len(nat)) int32."""
    pix = _planes(pix)
    C, H, W = pix.shape
    nat = np.ascontiguousarray(nat, dtype=np.int32)
    nb = C * (H // 8) * (W // 8)
    out = np.zeros((nb, len(nat)), np.int32)
    _lib().orc_q2_blocks(_ptr(pix), C, H, W, _ptr(nat), len(nat), _ptr(out))
    return out


def blocks_of(pix: np.ndarray) -> np.ndarray:
    """(nb, 64) pixel values in block order b = (c*By+by)*Bx+bx, p = 8y+x."""
    pix = _planes(pix)
    C, H, W = pix.shape
    return pix.reshape(C, H // 8, 8, W // 8, 8).transpose(0, 1, 3, 2, 4).reshape(-1, 64)


def tile_offset(nb: int, P: int, b: int, j: int) -> int:
    return int(_lib().orc_tile_offset(nb, P, b, j))


def tile_pack(vals: np.ndarray) -> np.ndarray:
    """(nb, P) block-major values -> flat tile-interleaved layout (oracle's own index math)."""
    nb, P = vals.shape
    out = np.empty(nb * P, vals.dtype)
    for t0 in range(0, nb, 64):
        nt = min(64, nb - t0)
        out[t0 * P:(t0 + nt) * P] = vals[t0:t0 + nt].T.reshape(-1)
    return out


def tile_unpack(flat: np.ndarray, nb: int, P: int) -> np.ndarray:
    """Inverse of tile_pack: flat tile layout -> (nb, P)."""
    out = np.empty((nb, P), flat.dtype)
    for t0 in range(0, nb, 64):
        nt = min(64, nb - t0)
        out[t0:t0 + nt] = flat[t0 * P:(t0 + nt) * P].reshape(P, nt).T
    return out


# ---------------------------------------------------------------- AES / CTR
def aes_sbox() -> np.ndarray:
    s = np.zeros(256, np.uint8)
    _lib().orc_aes_sbox(_ptr(s))
    return s


def aes_expand(key: bytes) -> bytes:
    k = np.frombuffer(bytes(key), np.uint8).copy()
    rk = np.zeros(176, np.uint8)
    _lib().orc_aes_expand(_ptr(k), _ptr(rk))
    return rk.tobytes()


def aes128_encrypt(key: bytes, block: bytes) -> bytes:
    k = np.frombuffer(bytes(key), np.uint8).copy()
    i = np.frombuffer(bytes(block), np.uint8).copy()
    o = np.zeros(16, np.uint8)
    _lib().orc_aes128_encrypt(_ptr(k), _ptr(i), _ptr(o))
    return o.tobytes()


def ctr_xor(key: bytes, ctr0: bytes, data, first_block: int = 0) -> np.ndarray:
    k = np.frombuffer(bytes(key), np.uint8).copy()
    c = np.frombuffer(bytes(ctr0), np.uint8).copy()
    d = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if isinstance(data, (bytes, bytearray)) else data, dtype=np.uint8)
    out = np.zeros_like(d)
    _lib().orc_ctr_xor(_ptr(k), _ptr(c), first_block, _ptr(d), _ptr(out), d.size)
    return out


def ctr_keystream(key: bytes, ctr0: bytes, block_indices) -> np.ndarray:
    """(n, 16) keystream blocks E_K(ctr0 + i) for the given block indices."""
    k = np.frombuffer(bytes(key), np.uint8).copy()
    c = np.frombuffer(bytes(ctr0), np.uint8).copy()
    idx = np.ascontiguousarray(block_indices, dtype=np.uint64)
    out = np.zeros((idx.size, 16), np.uint8)
    _lib().orc_ctr_keystream(_ptr(k), _ptr(c), _ptr(idx), idx.size, _ptr(out))
    return out


def tile_offsets(nb: int, P: int, blocks, j) -> np.ndarray:
    """Vector form of tile_offset (same index formula) for arrays of blocks / values."""
    b = np.asarray(blocks, np.int64)
    t = b // 64
    nt = np.minimum(64, nb - 64 * t)
    return 64 * t * P + np.asarray(j, np.int64) * nt + b % 64


# ---------------------------------------------------------------- pipeline
def popcount(mask: int) -> int:
    return bin(mask & ((1 << 64) - 1)).count("1")


def prefix_mask(k: int) -> int:
    """DC plus the first k zigzag AC coefficients."""
    return (1 << (k + 1)) - 1


def frag(pix: np.ndarray, mask: int, key: bytes | None = None, ctr0: bytes | None = None, exc_cap: int = 1 << 20):
    """Oracle fragmentation.  Returns dict with
    public (flat float64, tile layout), private (flat int16, tile layout),
    cipher (uint8 bytes or None), exc_index/exc_value (FP64 exceptions),
    max_err (largest FP64 |IDCT(stored) - x|)."""
    pix = _planes(pix)
    C, H, W = pix.shape
    nb = C * (H // 8) * (W // 8)
    npriv = popcount(mask)
    pub = np.zeros(nb * (64 - npriv), np.float64)
    priv = np.zeros(nb * npriv, np.int16)
    cipher = np.zeros(2 * nb * npriv, np.uint8) if key is not None else None
    exc_i = np.zeros(exc_cap, np.int64)
    exc_v = np.zeros(exc_cap, np.uint8)
    maxerr = np.zeros(1, np.float64)
    k = np.frombuffer(bytes(key), np.uint8).copy() if key is not None else None
    c = np.frombuffer(bytes(ctr0), np.uint8).copy() if key is not None else None
    n = _lib().orc_frag(_ptr(pix), C, H, W, mask, _ptr(pub), _ptr(priv),
                        _ptr(k) if k is not None else None, _ptr(c) if c is not None else None,
                        _ptr(cipher) if cipher is not None else None,
                        _ptr(exc_i), _ptr(exc_v), exc_cap, _ptr(maxerr))
    if n < 0:
        raise ValueError("private coefficient outside int16")
    if n > exc_cap:
        raise ValueError("exception capacity too small: %d" % n)
    return dict(public=pub, private=priv, cipher=cipher, exc_index=exc_i[:n].copy(),
                exc_value=exc_v[:n].copy(), max_err=float(maxerr[0]), nb=nb, npriv=npriv)


def defrag(shape, mask: int, public: np.ndarray, private: np.ndarray | None = None, key: bytes | None = None,
           ctr0: bytes | None = None, cipher: np.ndarray | None = None, exc_index=None, exc_value=None) -> np.ndarray:
    """Oracle defragmentation -> uint8 planes of ``shape`` (C, H, W)."""
    C, H, W = shape
    pub = np.ascontiguousarray(public, dtype=np.float64)
    out = np.zeros((C, H, W), np.uint8)
    ei = np.ascontiguousarray(exc_index if exc_index is not None else np.zeros(0), dtype=np.int64)
    ev = np.ascontiguousarray(exc_value if exc_value is not None else np.zeros(0), dtype=np.uint8)
    pr = np.ascontiguousarray(private, dtype=np.int16) if private is not None else None
    k = np.frombuffer(bytes(key), np.uint8).copy() if key is not None else None
    c = np.frombuffer(bytes(ctr0), np.uint8).copy() if key is not None else None
    ci = np.ascontiguousarray(cipher, dtype=np.uint8) if cipher is not None else None
    _lib().orc_defrag(C, H, W, mask, _ptr(pub), _ptr(pr) if pr is not None else None,
                      _ptr(k) if k is not None else None, _ptr(c) if c is not None else None,
                      _ptr(ci) if ci is not None else None, _ptr(ei), _ptr(ev), ei.size, _ptr(out))
    return out


# ---------------------------------------------------------------- soft mask (FP64)
def sigmoid(l):
    return 1.0 / (1.0 + np.exp(-np.asarray(l, np.float64)))


def _img_blocks(x: np.ndarray) -> np.ndarray:
    """(H, W) -> (nb, 64) block-major."""
    H, W = x.shape
    return x.reshape(H // 8, 8, W // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)


def _img_unblocks(b: np.ndarray, H: int, W: int) -> np.ndarray:
    return b.reshape(H // 8, W // 8, 8, 8).transpose(0, 2, 1, 3).reshape(H, W)


def softmask_public(x: np.ndarray, logits: np.ndarray) -> np.ndarray:
    """Public image of a soft frequency mask: P = IDCT(DCT(x) * (1 - sigmoid(l))) per 8x8 block.
    x: (B, H, W); logits: 64 values in natural (u, v) order.  The hard-mask
    case is the zero-padded public image of Sec. 6.3.1 (Fig. 7b)."""
    x = np.asarray(x, np.float64)
    Bm = basis()
    keep = 1.0 - sigmoid(logits)
    out = np.empty_like(x)
    for i in range(x.shape[0]):
        blk = _img_blocks(x[i])
        coef = blk @ Bm.T
        out[i] = _img_unblocks((coef * keep[None, :]) @ Bm, *x.shape[1:])
    return out


def pearson(a: np.ndarray, b: np.ndarray) -> float:
    """Correlation coefficient of Sec. 6.6.2: cov(a,b) / sqrt(D(a) D(b)), population moments."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    ma, mb = a.mean(), b.mean()
    cov = ((a - ma) * (b - mb)).mean()
    return float(cov / np.sqrt(((a - ma) ** 2).mean() * ((b - mb) ** 2).mean()))


LAMBDA = 0.1
BUDGET = 6.0


def softmask_loss(x: np.ndarray, logits: np.ndarray, lam: float = LAMBDA, budget: float = BUDGET) -> float:
    """L = mean_b rho(P_b, x_b)^2 + lam * (sum_n m_n - budget)^2."""
    P = softmask_public(x, logits)
    rho = np.array([pearson(P[i], x[i]) for i in range(x.shape[0])])
    m = sigmoid(logits)
    return float((rho ** 2).mean() + lam * (m.sum() - budget) ** 2)


def softmask_grad(x: np.ndarray, logits: np.ndarray, lam: float = LAMBDA, budget: float = BUDGET):
    """dL/dlogits by the adjoint route:
      G = dL/dP (closed form of the Pearson derivative),
      dL/dm_n = - sum_{images, blocks} DCT(G)_n * DCT(x)_n,
      dL/dl_n = sigmoid'(l_n) * (dL/dm_n + 2 lam (sum m - budget)).
    Returns (grad, loss, rho)."""
    x = np.asarray(x, np.float64)
    Bimg, H, W = x.shape
    N = H * W
    Bm = basis()
    m = sigmoid(logits)
    keep = 1.0 - m
    dm = np.zeros(64)
    rhos = np.zeros(Bimg)
    for i in range(Bimg):
        blk = _img_blocks(x[i])
        X = blk @ Bm.T
        Pb = (X * keep[None, :]) @ Bm
        xm, pm = blk.mean(), Pb.mean()
        sx = np.sqrt(((blk - xm) ** 2).mean())
        sp = np.sqrt(((Pb - pm) ** 2).mean())
        rho = ((blk - xm) * (Pb - pm)).mean() / (sx * sp)
        rhos[i] = rho
        # d(rho^2 / B)/dP
        G = (2.0 * rho / Bimg) * ((blk - xm) / (sx * sp) - rho * (Pb - pm) / sp ** 2) / N
        Ghat = G @ Bm.T
        dm -= (Ghat * X).sum(0)
    loss = float((rhos ** 2).mean() + lam * (m.sum() - budget) ** 2)
    grad = m * (1.0 - m) * (dm + 2.0 * lam * (m.sum() - budget))
    return grad, loss, rhos


def softmask_stats(x: np.ndarray):
    """Per image: E_n = sum over blocks of DCT(x)_n^2 (64 values, natural
    order) and the sample sum; the statistics the closed-form loss needs."""
    x = np.asarray(x, np.float64)
    Bm = basis()
    E = np.empty((x.shape[0], 64))
    sx = np.empty(x.shape[0])
    for i in range(x.shape[0]):
        blk = _img_blocks(x[i])
        E[i] = ((blk @ Bm.T) ** 2).sum(0)
        sx[i] = blk.sum()
    return E, sx


def softmask_adam(x: np.ndarray, logits: np.ndarray, steps: int, lr: float, lam: float = LAMBDA,
                  budget: float = BUDGET):
    """Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the logits with the adjoint
    gradient of softmask_grad.  Returns (logits, loss before each step)."""
    l = np.array(logits, np.float64)
    mom = np.zeros(64)
    vel = np.zeros(64)
    trace = []
    for t in range(1, steps + 1):
        g, loss, _ = softmask_grad(x, l, lam, budget)
        trace.append(loss)
        mom = 0.9 * mom + 0.1 * g
        vel = 0.999 * vel + 0.001 * g * g
        l = l - lr * (mom / (1 - 0.9 ** t)) / (np.sqrt(vel / (1 - 0.999 ** t)) + 1e-8)
    return l, np.array(trace)


def harden(logits: np.ndarray, n_private: int) -> int:
    """private_mask of the n_private largest logits (ties to the lower natural
    index): logit n belongs to natural frequency n, and the mask has bit z set
    for the zigzag position z of each chosen frequency."""
    order = sorted(range(64), key=lambda n: (-float(logits[n]), n))
    pos = np.empty(64, np.int64)
    pos[zigzag()] = np.arange(64)
    return sum(1 << int(pos[n]) for n in order[:n_private])


def softmask_adjoint(x: np.ndarray, G: np.ndarray, logits: np.ndarray) -> np.ndarray:
    """Gradient of the linear functional <G, P(logits)> with respect to the
    logits: sigmoid'(l_n) * (- sum over images and blocks of DCT(G)_n DCT(x)_n),
    the transposed transform applied to G."""
    x = np.asarray(x, np.float64)
    G = np.asarray(G, np.float64)
    Bm = basis()
    acc = np.zeros(64)
    for i in range(x.shape[0]):
        acc += ((_img_blocks(G[i]) @ Bm.T) * (_img_blocks(x[i]) @ Bm.T)).sum(0)
    m = sigmoid(logits)
    return m * (1.0 - m) * -acc
