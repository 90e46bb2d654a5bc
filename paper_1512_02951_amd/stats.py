"""Binding of the security statistics (sf_stats_workspace_bytes /
sf_security_stats_compute): argument marshalling and buffer allocation with
torch only; every statistic is computed by the HIP library."""
from __future__ import annotations

import ctypes

from . import check, lib as _base_lib, _stream

DIRS = ("h", "v", "d")


class SfSecurityStats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_uint64), ("hist_x", ctypes.c_uint64 * 256), ("hist_y", ctypes.c_uint64 * 256),
                ("pair_x", (ctypes.c_uint64 * 6) * 3), ("pair_y", (ctypes.c_uint64 * 6) * 3),
                ("cross", ctypes.c_uint64 * 6), ("bits_differing", ctypes.c_uint64), ("chi2_y", ctypes.c_double),
                ("entropy_x", ctypes.c_double), ("entropy_y", ctypes.c_double), ("joint_entropy", ctypes.c_double),
                ("mutual_information", ctypes.c_double), ("nmi", ctypes.c_double),
                ("corr_x", ctypes.c_double * 3), ("corr_y", ctypes.c_double * 3), ("corr2", ctypes.c_double),
                ("dif", ctypes.c_double), ("psnr", ctypes.c_double), ("block_entropy_x", ctypes.c_double * 4),
                ("block_entropy_y", ctypes.c_double * 4)]


def _declare(L):
    P = ctypes.c_void_p
    L.sf_stats_workspace_bytes.argtypes = []
    L.sf_stats_workspace_bytes.restype = ctypes.c_size_t
    L.sf_security_stats_compute.argtypes = [P, P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P,
                                            ctypes.c_size_t, P, P, P]
    L.sf_security_stats_compute.restype = ctypes.c_int


_declared = False


def lib():
    global _declared
    L = _base_lib()
    if not _declared:
        _declare(L)
        _declared = True
    return L


class StatsRunner:
    """Holds the device workspace and output record for repeated calls."""

    def __init__(self, device):
        import torch
        L = lib()
        self.ws = torch.empty(L.sf_stats_workspace_bytes(), dtype=torch.uint8, device=device)
        self.out = torch.empty(ctypes.sizeof(SfSecurityStats), dtype=torch.uint8, device=device)

    def launch(self, x, y, block_entropy=None, stream=None):
        if x.dim() == 2:
            x, y = x.unsqueeze(0), y.unsqueeze(0)
        assert x.shape == y.shape and x.is_contiguous() and y.is_contiguous()
        C, H, W = x.shape
        be = ctypes.c_void_p(block_entropy.data_ptr()) if block_entropy is not None else None
        check(lib().sf_security_stats_compute(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), H, W, C,
                                              ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                              ctypes.c_void_p(self.out.data_ptr()), be, _stream(stream)))

    def result(self) -> dict:
        """Copy the record to the host (synchronises) and return it as a dict."""
        raw = bytes(self.out.cpu().numpy().tobytes())
        r = SfSecurityStats.from_buffer_copy(raw)
        d = {f: getattr(r, f) for f, _ in SfSecurityStats._fields_}
        d["hist_x"], d["hist_y"] = list(r.hist_x), list(r.hist_y)
        for im in ("x", "y"):
            pm = getattr(r, "pair_" + im)
            for k, dname in enumerate(DIRS):
                d["moments_%s_%s" % (im, dname)] = tuple(int(v) for v in pm[k])
                d["corr_%s_%s" % (im, dname)] = getattr(r, "corr_" + im)[k]
            d["block_entropy_" + im] = list(getattr(r, "block_entropy_" + im))
        d["cross"] = tuple(int(v) for v in r.cross)
        for k in ("pair_x", "pair_y", "corr_x", "corr_y"):
            del d[k]
        return d

    def joint_histogram(self):
        """(256, 256) joint histogram left in the workspace by the last call."""
        return self.ws[:65536 * 4].view(dtype=__import__("torch").int32).view(256, 256)


def security_stats(x, y, block_entropy: bool = False, stream=None):
    """Statistics of protected y against original x (uint8 CUDA tensors,
    same (C, H, W) shape).  Returns (dict, block entropies or None)."""
    import torch
    r = StatsRunner(x.device)
    be = None
    if block_entropy:
        C, H, W = x.shape if x.dim() == 3 else (1,) + tuple(x.shape)
        be = torch.empty(2 * C * (H // 8) * (W // 8), dtype=torch.float32, device=x.device)
    r.launch(x, y, be, stream)
    return r.result(), be
