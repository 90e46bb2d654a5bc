"""MI355X (gfx950) selective fragmentation: thin Python binding of libsefrag.so.

Every step of the method runs in the HIP library; this module only marshals
arguments (device pointers of torch tensors, the current HIP stream) into the
C ABI declared in ``include/sefrag.h``.  PyTorch provides device memory and
streams.  If the compiled library is missing, :func:`lib` raises; there is no
fallback path.

Entry points (same names as the C ABI): :func:`frag_image`,
:func:`defrag_image`, :func:`encrypt_private`, :func:`fragment_sizes`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsefrag.so")

SF_OK, SF_EINVAL, SF_ESHAPE, SF_ERANGE, SF_EHIP, SF_ENOTSUP = 0, -1, -2, -3, -5, -6
SF_STATUS_EXC_OVERFLOW, SF_STATUS_RESIDUAL_RANGE, SF_STATUS_PRIVATE_RANGE = 1, 2, 4
SF_FP32, SF_FP16, SF_BF16 = 0, 1, 2
PRECISIONS = {"fp32": SF_FP32, "fp16": SF_FP16, "bf16": SF_BF16}


class SfDesc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_uint32), ("width", ctypes.c_uint32), ("channels", ctypes.c_uint32),
                ("precision", ctypes.c_uint32), ("private_mask", ctypes.c_uint64)]


class SfAesCtr(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint8 * 16), ("ctr0", ctypes.c_uint8 * 16)]


class SfExceptions(ctypes.Structure):
    _fields_ = [("d_buf", ctypes.c_void_p), ("per_tile", ctypes.c_uint32)]


class SfLaunchShape(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_uint32), ("resident", ctypes.c_uint32)]


class SefragError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("sefrag error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libsefrag.so (build it with paper_1512_02951_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsefrag.so is not built; run python -m paper_1512_02951_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
        L.sf_version.restype = ctypes.c_char_p
        L.sf_strerror.restype = ctypes.c_char_p
        L.sf_strerror.argtypes = [i32]
        L.sf_last_error.restype = ctypes.c_char_p
        L.sf_fragment_sizes.argtypes = [ctypes.POINTER(SfDesc), ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.sf_exception_bytes.argtypes = [ctypes.POINTER(SfDesc), u32, ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_int)]
        L.sf_init.argtypes = []
        L.frag_image.argtypes = [ctypes.POINTER(SfDesc), P, P, P, ctypes.POINTER(SfExceptions), P,
                                 ctypes.POINTER(SfAesCtr), P, P]
        L.defrag_image.argtypes = [ctypes.POINTER(SfDesc), P, P, ctypes.POINTER(SfExceptions), P,
                                   ctypes.POINTER(SfAesCtr), P, P, P]
        L.encrypt_private.argtypes = [ctypes.POINTER(SfAesCtr), u64, P, P, sz, P]
        L.sf_set_launch_shape.argtypes = [ctypes.POINTER(SfDesc), i32, ctypes.POINTER(SfLaunchShape)]
        L.sf_get_launch_shape.argtypes = [ctypes.POINTER(SfDesc), i32, ctypes.POINTER(SfLaunchShape)]
        L.sf_tune_image.argtypes = [ctypes.POINTER(SfDesc), P, P, P, ctypes.POINTER(SfExceptions), P,
                                    ctypes.POINTER(SfAesCtr), P, P, P, ctypes.POINTER(SfLaunchShape),
                                    ctypes.POINTER(SfLaunchShape), ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(ctypes.c_float)]
        for name in ("sf_fragment_sizes", "sf_exception_bytes", "sf_init", "frag_image", "defrag_image",
                     "encrypt_private", "sf_set_launch_shape", "sf_get_launch_shape", "sf_tune_image"):
            getattr(L, name).restype = i32
        _extend(L)
        _lib = L
    return _lib


_extensions = []


def _extend(L):
    for f in _extensions:
        f(L)


def check(rc: int) -> None:
    if rc != SF_OK:
        raise SefragError(rc, lib().sf_last_error().decode() or lib().sf_strerror(rc).decode())


def desc(H: int, W: int, C: int, mask: int, precision="fp32") -> SfDesc:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return SfDesc(H, W, C, p, mask & ((1 << 64) - 1))


def aes_ctr(key: bytes | None, ctr0: bytes | None):
    if key is None:
        return None
    a = SfAesCtr()
    a.key[:] = list(bytes(key))
    a.ctr0[:] = list(bytes(ctr0 if ctr0 is not None else bytes(16)))
    return a


def fragment_sizes(H: int, W: int, C: int, mask: int, precision="fp32"):
    """(public_bytes, private_bytes, residual_bytes) for an image; host only."""
    d = desc(H, W, C, mask, precision)
    pb, qb, rb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().sf_fragment_sizes(ctypes.byref(d), ctypes.byref(pb), ctypes.byref(qb), ctypes.byref(rb)))
    return pb.value, qb.value, rb.value


def prefix_mask(k: int) -> int:
    """DC plus the first k zigzag AC coefficients."""
    return (1 << (k + 1)) - 1


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def exception_bytes(H: int, W: int, C: int, mask: int, per_tile: int, precision="fp32"):
    """(bytes, needed) of an exception buffer; host only."""
    d = desc(H, W, C, mask, precision)
    nbytes, needed = ctypes.c_size_t(), ctypes.c_int()
    check(lib().sf_exception_bytes(ctypes.byref(d), per_tile, ctypes.byref(nbytes), ctypes.byref(needed)))
    return nbytes.value, bool(needed.value)


DEFAULT_PER_TILE = 64


@dataclass
class ExceptionList:
    """Per-tile exception slots (one device byte buffer): samples the plain
    form cannot restore from its fragments, and the samples whose residual
    the reduced-precision forms cannot code in 2 bits."""
    buf: "object"
    per_tile: int
    shape: tuple

    @staticmethod
    def empty(shape, mask: int, per_tile: int = DEFAULT_PER_TILE, device="cuda", precision="fp32"):
        import torch
        C, H, W = shape
        nbytes, needed = exception_bytes(H, W, C, mask, per_tile, precision)
        buf = torch.zeros(max(nbytes, 16), dtype=torch.uint8, device=device) if needed else None
        return ExceptionList(buf, per_tile, tuple(shape))

    def c(self) -> SfExceptions:
        return SfExceptions(self.buf.data_ptr() if self.buf is not None else None, self.per_tile)

    def decode(self):
        """Host copy of the entries: (sample indices, values, counts per tile)."""
        import numpy as np
        C, H, W = self.shape
        nb = C * H * W // 64
        nt = (nb + 63) // 64
        if self.buf is None:
            return np.zeros(0, np.int64), np.zeros(0, np.uint8), np.zeros(nt, np.int64)
        raw = self.buf.cpu().numpy()
        a16 = lambda v: (v + 15) // 16 * 16
        pos_off = a16(2 * nt)
        val_off = pos_off + a16(2 * nt * self.per_tile)
        counts = raw[:2 * nt].view("<u2").astype(np.int64)
        pos = raw[pos_off:pos_off + 2 * nt * self.per_tile].view("<u2").reshape(nt, self.per_tile)
        val = raw[val_off:val_off + nt * self.per_tile].reshape(nt, self.per_tile)
        Bx, By = W // 8, H // 8
        idx, vals = [], []
        for t in np.flatnonzero(counts):
            for e in range(min(counts[t], self.per_tile)):
                b = 64 * t + int(pos[t, e]) // 64
                p = int(pos[t, e]) % 64
                c, rem = divmod(b, Bx * By)
                by, bx = divmod(rem, Bx)
                idx.append(c * H * W + (8 * by + p // 8) * W + 8 * bx + p % 8)
                vals.append(val[t, e])
        return np.array(idx, np.int64), np.array(vals, np.uint8), counts


@dataclass
class Fragments:
    public: "object"
    private: "object"
    exceptions: ExceptionList | None
    residual: "object"
    shape: tuple
    mask: int
    precision: str


def frag_image(pixels, mask: int, key: bytes | None = None, ctr0: bytes | None = None, precision="fp32",
               out: Fragments | None = None, status=None, stream=None) -> Fragments:
    """Fragment a uint8 CUDA tensor (C, H, W) (or (H, W)).  Output buffers are
    allocated with torch unless ``out`` supplies them."""
    import torch
    if pixels.dim() == 2:
        pixels = pixels.unsqueeze(0)
    assert pixels.dtype == torch.uint8 and pixels.is_cuda and pixels.is_contiguous()
    C, H, W = pixels.shape
    prec = precision if isinstance(precision, str) else {v: k for k, v in PRECISIONS.items()}[precision]
    pb, qb, rb = fragment_sizes(H, W, C, mask, prec)
    if out is None:
        pub_dtype = torch.float32 if prec == "fp32" else (torch.float16 if prec == "fp16" else torch.bfloat16)
        esz = 4 if prec == "fp32" else 2
        out = Fragments(
            public=torch.empty(max(pb // esz, 1), dtype=pub_dtype, device=pixels.device),
            private=torch.empty(max(qb, 16), dtype=torch.uint8, device=pixels.device),
            exceptions=ExceptionList.empty((C, H, W), mask, device=pixels.device, precision=prec),
            residual=torch.empty(rb, dtype=torch.uint8, device=pixels.device) if rb else None,
            shape=(C, H, W), mask=mask, precision=prec)
    d = desc(H, W, C, mask, prec)
    exc = out.exceptions.c() if out.exceptions is not None else None
    rc = lib().frag_image(ctypes.byref(d), _ptr(pixels), _ptr(out.public), _ptr(out.private),
                          ctypes.byref(exc) if exc is not None else None, _ptr(out.residual),
                          ctypes.byref(aes_ctr(key, ctr0)) if key is not None else None,
                          _ptr(status), _stream(stream))
    check(rc)
    return out


def defrag_image(frags: Fragments, key: bytes | None = None, ctr0: bytes | None = None, out=None, status=None,
                 stream=None):
    """Defragment; returns the uint8 CUDA tensor (C, H, W)."""
    import torch
    C, H, W = frags.shape
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.uint8, device=frags.private.device)
    d = desc(H, W, C, frags.mask, frags.precision)
    exc = frags.exceptions.c() if frags.exceptions is not None else None
    rc = lib().defrag_image(ctypes.byref(d), _ptr(frags.public), _ptr(frags.private),
                            ctypes.byref(exc) if exc is not None else None, _ptr(frags.residual),
                            ctypes.byref(aes_ctr(key, ctr0)) if key is not None else None,
                            _ptr(out), _ptr(status), _stream(stream))
    check(rc)
    return out


WHICH = {"frag": 0, "defrag": 1}


def set_launch_shape(shape: tuple, mask: int, which: str, waves_per_group: int | None, resident: int = 0,
                     precision="fp32") -> None:
    """The launch shape frag_image / defrag_image use on the current device for
    images of this (C, H, W) size class, mask and precision; waves_per_group
    None forgets it."""
    C, H, W = shape
    d = desc(H, W, C, mask, precision)
    s = SfLaunchShape(waves_per_group, resident) if waves_per_group is not None else None
    check(lib().sf_set_launch_shape(ctypes.byref(d), WHICH[which], ctypes.byref(s) if s is not None else None))


def launch_shape(shape: tuple, mask: int, which: str, precision="fp32") -> tuple:
    """(waves_per_group, resident) that the next call would use."""
    C, H, W = shape
    d = desc(H, W, C, mask, precision)
    s = SfLaunchShape()
    check(lib().sf_get_launch_shape(ctypes.byref(d), WHICH[which], ctypes.byref(s)))
    return s.waves_per_group, s.resident


def tune_image(pixels, mask: int, key: bytes | None = None, ctr0: bytes | None = None, precision="fp32",
               out: Fragments | None = None, restored=None, status=None, stream=None) -> dict:
    """Times frag_image and defrag_image of ``pixels`` in every launch shape
    and keeps the fastest for this size class, mask and precision (sf_tune_image).
    Returns the shapes and their times; ``out`` and ``restored`` (allocated
    if None) hold the results of a round trip in those shapes."""
    import torch
    if pixels.dim() == 2:
        pixels = pixels.unsqueeze(0)
    C, H, W = pixels.shape
    if out is None:
        out = frag_image(pixels, mask, key, ctr0, precision=precision, status=status, stream=stream)
    if restored is None:
        restored = torch.empty_like(pixels)
    d = desc(H, W, C, mask, out.precision)
    exc = out.exceptions.c() if out.exceptions is not None else None
    bf, bd = SfLaunchShape(), SfLaunchShape()
    fm, dm = ctypes.c_float(), ctypes.c_float()
    check(lib().sf_tune_image(ctypes.byref(d), _ptr(pixels), _ptr(out.public), _ptr(out.private),
                              ctypes.byref(exc) if exc is not None else None, _ptr(out.residual),
                              ctypes.byref(aes_ctr(key, ctr0)) if key is not None else None, _ptr(restored),
                              _ptr(status), _stream(stream), ctypes.byref(bf), ctypes.byref(bd),
                              ctypes.byref(fm), ctypes.byref(dm)))
    return {"frag": (bf.waves_per_group, bf.resident), "defrag": (bd.waves_per_group, bd.resident),
            "frag_ms": fm.value, "defrag_ms": dm.value, "fragments": out, "restored": restored}


def encrypt_private(key: bytes, ctr0: bytes, data, out=None, first_block: int = 0, stream=None):
    """AES-128-CTR over a uint8 CUDA tensor (also decrypts)."""
    import torch
    assert data.dtype == torch.uint8 and data.is_cuda and data.is_contiguous()
    if out is None:
        out = torch.empty_like(data)
    a = aes_ctr(key, ctr0)
    check(lib().encrypt_private(ctypes.byref(a), first_block, _ptr(data), _ptr(out), data.numel(), _stream(stream)))
    return out
