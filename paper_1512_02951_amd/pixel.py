"""Binding of the pixel-domain formats (sf_pixel_fragment_sizes /
pixel_frag_image / pixel_defrag_image): argument marshalling and buffer
allocation with torch only; quantiser, packing, hashing, cipher and inverse
run in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import SfAesCtr, SfDesc, aes_ctr, check, desc, lib as _base_lib, _stream

SF_LEVEL_FIRST, SF_LEVEL_STRONG, SF_STORAGE_8BIT = 0, 1, 2


def _declare(L):
    P, i32 = ctypes.c_void_p, ctypes.c_int
    D, A, SZ = ctypes.POINTER(SfDesc), ctypes.POINTER(SfAesCtr), ctypes.POINTER(ctypes.c_size_t)
    L.sf_pixel_fragment_sizes.argtypes = [D, i32, SZ, SZ]
    L.pixel_frag_image.argtypes = [D, i32, P, P, P, A, P]
    L.pixel_defrag_image.argtypes = [D, i32, P, P, A, P, P]
    for n in ("sf_pixel_fragment_sizes", "pixel_frag_image", "pixel_defrag_image"):
        getattr(L, n).restype = i32


_declared = False


def lib():
    global _declared
    L = _base_lib()
    if not _declared:
        _declare(L)
        _declared = True
    return L


def _flags(strong: bool, storage_bits: int) -> int:
    assert storage_bits in (8, 11)
    return (SF_LEVEL_STRONG if strong else SF_LEVEL_FIRST) | (SF_STORAGE_8BIT if storage_bits == 8 else 0)


def fragment_sizes(H: int, W: int, C: int, mask: int, strong: bool = False, storage_bits: int = 11):
    """(public_bytes, private_bytes); host only."""
    d = desc(H, W, C, mask)
    pb, qb = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().sf_pixel_fragment_sizes(ctypes.byref(d), _flags(strong, storage_bits), ctypes.byref(pb),
                                        ctypes.byref(qb)))
    return pb.value, qb.value


@dataclass
class PixelFragments:
    public: "object"    # uint8 CUDA tensor (C, H, W)
    private: "object"   # uint8 CUDA tensor, packed fields (ciphertext when keyed)
    mask: int
    strong: bool
    shape: tuple
    storage_bits: int = 11


def _aes(key, ctr0):
    a = aes_ctr(key, ctr0)
    return ctypes.byref(a) if a is not None else None


def pixel_frag_image(pixels, mask: int, strong: bool = False, key: bytes | None = None, ctr0: bytes | None = None,
                     out: PixelFragments | None = None, stream=None, storage_bits: int = 11) -> PixelFragments:
    """Fragment a uint8 CUDA tensor (C, H, W) (or (H, W)); storage_bits 11
    (exact) or 8 (the report's lossy storage)."""
    import torch
    if pixels.dim() == 2:
        pixels = pixels.unsqueeze(0)
    assert pixels.dtype == torch.uint8 and pixels.is_cuda and pixels.is_contiguous()
    C, H, W = pixels.shape
    d = desc(H, W, C, mask)
    _, qb = fragment_sizes(H, W, C, mask, strong, storage_bits)
    if out is None:
        out = PixelFragments(torch.empty((C, H, W), dtype=torch.uint8, device=pixels.device),
                             torch.empty(max(qb, 16), dtype=torch.uint8, device=pixels.device), mask, strong,
                             (C, H, W), storage_bits)
    else:
        assert out.public.numel() >= C * H * W and out.private.numel() >= qb, "fragment buffers too small"
        out.mask, out.strong, out.shape, out.storage_bits = mask, strong, (C, H, W), storage_bits
    check(lib().pixel_frag_image(ctypes.byref(d), _flags(strong, storage_bits),
                                 ctypes.c_void_p(pixels.data_ptr()), ctypes.c_void_p(out.public.data_ptr()),
                                 ctypes.c_void_p(out.private.data_ptr()), _aes(key, ctr0), _stream(stream)))
    return out


def pixel_defrag_image(frags: PixelFragments, key: bytes | None = None, ctr0: bytes | None = None, out=None,
                       stream=None):
    """Defragment; returns the uint8 CUDA tensor (C, H, W)."""
    import torch
    C, H, W = frags.shape
    d = desc(H, W, C, frags.mask)
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.uint8, device=frags.public.device)
    check(lib().pixel_defrag_image(ctypes.byref(d), _flags(frags.strong, frags.storage_bits),
                                   ctypes.c_void_p(frags.public.data_ptr()), ctypes.c_void_p(frags.private.data_ptr()),
                                   _aes(key, ctr0), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out
