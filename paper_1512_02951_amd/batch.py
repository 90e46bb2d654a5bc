"""Binding of the batched form (sf_batch_plan / sf_frag_batch / sf_defrag_batch /
sf_batch_autotune): argument marshalling and buffer allocation with torch only.

A :class:`Batch` owns the fragments of a list of images and a planned device
workspace; :meth:`Batch.frag` / :meth:`Batch.defrag` enqueue one persistent
kernel each (plus a counter reset for the work-queue schedule) and can be
captured into a HIP graph.  The tuner's
choice can be cached in a small JSON file keyed by device and batch shape.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

from . import DEFAULT_PER_TILE, check, exception_bytes, fragment_sizes, lib as _base_lib, _stream


class SfBatchItem(ctypes.Structure):
    _fields_ = [("height", ctypes.c_uint32), ("width", ctypes.c_uint32), ("channels", ctypes.c_uint32),
                ("exc_per_tile", ctypes.c_uint32), ("private_mask", ctypes.c_uint64),
                ("d_pixels", ctypes.c_void_p), ("d_restored", ctypes.c_void_p), ("d_public", ctypes.c_void_p),
                ("d_private", ctypes.c_void_p), ("d_exc", ctypes.c_void_p), ("ctr0", ctypes.c_uint8 * 16)]


class SfBatchTuning(ctypes.Structure):
    _fields_ = [("tiles_per_grab", ctypes.c_uint32), ("workgroups_per_cu", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


SCHED_QUEUE, SCHED_STATIC = 0, 1


def _declare(L):
    P, u32, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int
    L.sf_batch_workspace_bytes.argtypes = [u32]
    L.sf_batch_workspace_bytes.restype = sz
    L.sf_batch_plan.argtypes = [ctypes.POINTER(SfBatchItem), u32, P, P, sz, P]
    L.sf_frag_batch.argtypes = [P, ctypes.POINTER(SfBatchTuning), P, P]
    L.sf_defrag_batch.argtypes = [P, ctypes.POINTER(SfBatchTuning), P, P]
    L.sf_batch_autotune.argtypes = [P, ctypes.POINTER(SfBatchTuning), ctypes.POINTER(ctypes.c_float), P]
    for n in ("sf_batch_plan", "sf_frag_batch", "sf_defrag_batch", "sf_batch_autotune"):
        getattr(L, n).restype = i32


_declared = False


def lib():
    """The shared library with the batch entry points declared."""
    global _declared
    L = _base_lib()
    if not _declared:
        _declare(L)
        _declared = True
    return L


class Batch:
    """Fragments of a batch of uint8 CUDA images (C, H, W) with per-image
    selections and counter blocks, and the planned device workspace."""

    def __init__(self, images, masks, key: bytes | None, ctr0s, per_tile: int = DEFAULT_PER_TILE, stream=None):
        import torch
        assert len(images) == len(masks) == len(ctr0s) and len(images) > 0
        self.images = images
        self.masks = list(masks)
        self.key = key
        self.publics, self.privates, self.excs, self.restored = [], [], [], []
        items = (SfBatchItem * len(images))()
        for i, (x, m, c0) in enumerate(zip(images, masks, ctr0s)):
            assert x.dtype == torch.uint8 and x.is_cuda and x.is_contiguous() and x.dim() == 3
            C, H, W = x.shape
            pb, qb, _ = fragment_sizes(H, W, C, m)
            eb, needed = exception_bytes(H, W, C, m, per_tile)
            pub = torch.empty(max(pb // 4, 1), dtype=torch.float32, device=x.device)
            prv = torch.empty(max(qb, 16), dtype=torch.uint8, device=x.device)
            exc = torch.zeros(max(eb, 16), dtype=torch.uint8, device=x.device) if needed else None
            out = torch.empty_like(x)
            self.publics.append(pub)
            self.privates.append(prv)
            self.excs.append(exc)
            self.restored.append(out)
            it = items[i]
            it.height, it.width, it.channels, it.exc_per_tile = H, W, C, per_tile
            it.private_mask = m & ((1 << 64) - 1)
            it.d_pixels, it.d_restored = x.data_ptr(), out.data_ptr()
            it.d_public, it.d_private = pub.data_ptr(), prv.data_ptr()
            it.d_exc = exc.data_ptr() if exc is not None else None
            it.ctr0[:] = list(bytes(c0))
        self.items = items
        ws_bytes = lib().sf_batch_workspace_bytes(len(images))
        self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=images[0].device)
        keybuf = (ctypes.c_uint8 * 16)(*bytes(key)) if key is not None else None
        check(lib().sf_batch_plan(items, len(images), keybuf, ctypes.c_void_p(self.workspace.data_ptr()), ws_bytes,
                                  _stream(stream)))
        self.tuning = None

    def _tuning(self, tuning):
        t = tuning if tuning is not None else self.tuning
        if t is None:
            return None
        if isinstance(t, SfBatchTuning):
            return ctypes.byref(t)
        # (tiles_per_grab, workgroups_per_cu[, schedule])
        return ctypes.byref(SfBatchTuning(int(t[0]), int(t[1]), int(t[2]) if len(t) > 2 else SCHED_QUEUE))

    def frag(self, tuning=None, status=None, stream=None):
        check(lib().sf_frag_batch(ctypes.c_void_p(self.workspace.data_ptr()), self._tuning(tuning),
                                  ctypes.c_void_p(status.data_ptr()) if status is not None else None, _stream(stream)))

    def defrag(self, tuning=None, status=None, stream=None):
        check(lib().sf_defrag_batch(ctypes.c_void_p(self.workspace.data_ptr()), self._tuning(tuning),
                                    ctypes.c_void_p(status.data_ptr()) if status is not None else None, _stream(stream)))

    def signature(self) -> str:
        """Shape class of the batch: image count, total samples and the selection mix."""
        tot = sum(x.numel() for x in self.images)
        mix = sorted(set(self.masks))
        return "n%d_s%d_m%s" % (len(self.images), tot, hashlib.sha1(repr(mix).encode()).hexdigest()[:8])

    def autotune(self, cache: str | None = None, stream=None):
        """Pick (tiles_per_grab, workgroups_per_cu, schedule) with the library's
        tuner; reuse a cached choice for the same device and batch signature."""
        import torch
        dev = torch.cuda.get_device_properties(self.workspace.device)
        key = "%s|%s" % (getattr(dev, "gcnArchName", dev.name), self.signature())
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            e = table[key]
            self.tuning = (e["tiles_per_grab"], e["workgroups_per_cu"], e.get("schedule", SCHED_QUEUE))
            return self.tuning, e.get("ms")
        best, ms = SfBatchTuning(), ctypes.c_float()
        check(lib().sf_batch_autotune(ctypes.c_void_p(self.workspace.data_ptr()), ctypes.byref(best),
                                      ctypes.byref(ms), _stream(stream)))
        self.tuning = (best.tiles_per_grab, best.workgroups_per_cu, best.schedule)
        if cache:
            table[key] = {"tiles_per_grab": best.tiles_per_grab, "workgroups_per_cu": best.workgroups_per_cu,
                          "schedule": best.schedule, "ms": ms.value}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return self.tuning, ms.value
