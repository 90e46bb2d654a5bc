"""Binding of the wavelet variant (dwt_frag_image / dwt_defrag_image /
sf_dwt_fragment_sizes): argument marshalling and buffer allocation with torch
only; the transform, split and cipher run in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import SfAesCtr, aes_ctr, check, lib as _base_lib, _stream


def _declare(L):
    P, u32, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int
    L.sf_dwt_fragment_sizes.argtypes = [u32, u32, u32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.dwt_frag_image.argtypes = [u32, u32, u32, P, P, P, ctypes.POINTER(SfAesCtr), P]
    L.dwt_defrag_image.argtypes = [u32, u32, u32, P, P, ctypes.POINTER(SfAesCtr), P, P]
    for n in ("sf_dwt_fragment_sizes", "dwt_frag_image", "dwt_defrag_image"):
        getattr(L, n).restype = i32


_declared = False


def lib():
    global _declared
    L = _base_lib()
    if not _declared:
        _declare(L)
        _declared = True
    return L


def fragment_sizes(H: int, W: int, C: int):
    """(public_bytes, private_bytes); host only."""
    pb, qb = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().sf_dwt_fragment_sizes(H, W, C, ctypes.byref(pb), ctypes.byref(qb)))
    return pb.value, qb.value


@dataclass
class DwtFragments:
    public: "object"    # int16 CUDA tensor, 60 values per block, tile layout
    private: "object"   # uint8 CUDA tensor (int16 little endian, ciphertext when keyed)
    shape: tuple


def _aes(key, ctr0):
    a = aes_ctr(key, ctr0)
    return ctypes.byref(a) if a is not None else None


def dwt_frag_image(pixels, key: bytes | None = None, ctr0: bytes | None = None, out: DwtFragments | None = None,
                   stream=None) -> DwtFragments:
    """Fragment a uint8 CUDA tensor (C, H, W) (or (H, W))."""
    import torch
    if pixels.dim() == 2:
        pixels = pixels.unsqueeze(0)
    assert pixels.dtype == torch.uint8 and pixels.is_cuda and pixels.is_contiguous()
    C, H, W = pixels.shape
    if out is None:
        pb, qb = fragment_sizes(H, W, C)
        out = DwtFragments(torch.empty(max(pb // 2, 8), dtype=torch.int16, device=pixels.device),
                           torch.empty(max(qb, 16), dtype=torch.uint8, device=pixels.device), (C, H, W))
    check(lib().dwt_frag_image(H, W, C, ctypes.c_void_p(pixels.data_ptr()), ctypes.c_void_p(out.public.data_ptr()),
                               ctypes.c_void_p(out.private.data_ptr()), _aes(key, ctr0), _stream(stream)))
    return out


def dwt_defrag_image(frags: DwtFragments, key: bytes | None = None, ctr0: bytes | None = None, out=None,
                     stream=None):
    """Defragment; returns the uint8 CUDA tensor (C, H, W)."""
    import torch
    C, H, W = frags.shape
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.uint8, device=frags.private.device)
    check(lib().dwt_defrag_image(H, W, C, ctypes.c_void_p(frags.public.data_ptr()),
                                 ctypes.c_void_p(frags.private.data_ptr()), _aes(key, ctr0),
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out
