"""CPU tests of the C ABI: the library loads, exports every declared symbol,
computes fragment sizes in closed form and rejects bad arguments before
touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_1512_02951_amd as sf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_loads_and_exports_every_declared_symbol():
    L = sf.lib()
    names = _declared_functions()
    assert {"frag_image", "defrag_image", "encrypt_private", "sf_fragment_sizes"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.sf_version()


@pytest.mark.parametrize("H,W,C,k,prec", [(512, 512, 1, 2, "fp32"), (4096, 4096, 3, 5, "fp32"),
                                          (8192, 8192, 1, 9, "fp16"), (8192, 8192, 1, 9, "bf16"),
                                          (8, 8, 1, 63, "fp32"), (24, 40, 3, 0, "fp32")])
def test_fragment_sizes_closed_form(H, W, C, k, prec):
    nb = H * W * C // 64
    npriv = k + 1
    pb, qb, rb = sf.fragment_sizes(H, W, C, sf.prefix_mask(k), prec)
    esz = 4 if prec == "fp32" else 2
    assert pb == nb * (64 - npriv) * esz
    assert qb == nb * npriv * 2
    assert rb == (0 if prec == "fp32" else H * W * C // 4)  # 2-bit residual codes


def test_workload_byte_counts():
    # 4096x4096 RGB, k = 5: 786432 blocks, 9437184 private bytes, 182452224 public bytes
    pb, qb, _ = sf.fragment_sizes(4096, 4096, 3, sf.prefix_mask(5))
    assert (pb, qb) == (182452224, 9437184)
    assert 2 * (4096 * 4096 * 3 + pb + qb) == 484442112


def _rc(fn, *args):
    return fn(*args)


@pytest.mark.parametrize("H,W,C,mask,prec,code", [
    (0, 8, 1, 1, 0, sf.SF_ESHAPE), (12, 8, 1, 1, 0, sf.SF_ESHAPE), (8, 20, 1, 1, 0, sf.SF_ESHAPE),
    (8, 8, 0, 1, 0, sf.SF_ESHAPE), (8, 8, 1, 0, 0, sf.SF_EINVAL), (8, 8, 1, 1, 7, sf.SF_EINVAL),
    (65536, 65536, 1, 1, 0, sf.SF_ESHAPE)])
def test_descriptor_validation(H, W, C, mask, prec, code):
    d = sf.SfDesc(H, W, C, prec, mask)
    L = sf.lib()
    out = ctypes.c_size_t()
    assert L.sf_fragment_sizes(ctypes.byref(d), ctypes.byref(out), None, None) == code
    assert L.sf_last_error()
    # frag/defrag validate before any device call
    exc = sf.SfExceptions(64, 1)
    assert L.frag_image(ctypes.byref(d), 64, 64, 64, ctypes.byref(exc), None, None, None, None) == code
    assert L.defrag_image(ctypes.byref(d), 64, 64, ctypes.byref(exc), None, None, 64, None, None) == code


def test_null_and_alignment_checks():
    L = sf.lib()
    d = sf.SfDesc(8, 8, 1, 0, 0x3F)
    exc = sf.SfExceptions(64, 4)
    assert L.frag_image(None, 64, 64, 64, ctypes.byref(exc), None, None, None, None) == sf.SF_EINVAL
    assert L.frag_image(ctypes.byref(d), None, 64, 64, ctypes.byref(exc), None, None, None, None) == sf.SF_EINVAL
    assert L.frag_image(ctypes.byref(d), 64, 64, 64, None, None, None, None, None) == sf.SF_EINVAL
    bad = sf.SfExceptions(64, 5000)
    assert L.frag_image(ctypes.byref(d), 64, 64, 64, ctypes.byref(bad), None, None, None, None) == sf.SF_ERANGE
    lp = sf.SfDesc(8, 8, 1, sf.SF_FP16, 0x3F)
    assert L.frag_image(ctypes.byref(lp), 64, 64, 64, None, None, None, None, None) == sf.SF_EINVAL  # no residual
    assert L.frag_image(ctypes.byref(d), 65, 64, 64, ctypes.byref(exc), None, None, None, None) == sf.SF_EINVAL
    assert L.frag_image(ctypes.byref(d), 64, 64, 72, ctypes.byref(exc), None, None, None, None) == sf.SF_EINVAL
    assert L.encrypt_private(None, 0, 64, 64, 16, None) == sf.SF_EINVAL
    a = sf.SfAesCtr()
    assert L.encrypt_private(ctypes.byref(a), 0, None, 64, 16, None) == sf.SF_EINVAL
    assert L.encrypt_private(ctypes.byref(a), 0, 64, 64, 0, None) == sf.SF_OK


def test_exception_buffer_layout_size():
    # 4096x4096 RGB: 12288 tiles; counts 24576 B, positions 2*12288*64, values 12288*64
    nbytes, needed = sf.exception_bytes(4096, 4096, 3, sf.prefix_mask(5), 64)
    assert needed and nbytes == 24576 + 2 * 12288 * 64 + 12288 * 64
    assert not sf.exception_bytes(4096, 4096, 3, sf.prefix_mask(4), 64)[1]
    with pytest.raises(sf.SefragError):
        sf.exception_bytes(64, 64, 1, 3, 4097)


def test_error_strings():
    L = sf.lib()
    for code in (sf.SF_OK, sf.SF_EINVAL, sf.SF_ESHAPE, sf.SF_ERANGE, sf.SF_EHIP, sf.SF_ENOTSUP):
        assert L.sf_strerror(code)


def test_c_consumer_builds_against_the_header(tmp_path):
    # a plain C program (tests/c_abi_roundtrip.c) compiles and links against
    # include/sefrag.h and the in-tree library; the GPU test runs it
    from c_abi_build import build_c_program
    assert os.path.exists(build_c_program(str(tmp_path)))


def test_launch_shape_arguments_are_checked_on_the_host():
    L = sf.lib()
    d = sf.SfDesc(64, 64, 1, 0, 0x3F)
    ok = sf.SfLaunchShape(2, 0)
    for which, shape in ((2, ok), (-1, ok), (0, sf.SfLaunchShape(3, 0)), (1, sf.SfLaunchShape(16, 0)),
                         (0, sf.SfLaunchShape(2, 2))):
        assert L.sf_set_launch_shape(ctypes.byref(d), which, ctypes.byref(shape)) == sf.SF_EINVAL
    assert L.sf_get_launch_shape(ctypes.byref(d), 0, None) == sf.SF_EINVAL
    bad = sf.SfDesc(12, 64, 1, 0, 0x3F)
    assert L.sf_set_launch_shape(ctypes.byref(bad), 0, ctypes.byref(ok)) == sf.SF_ESHAPE
    exc = sf.SfExceptions(64, 4)
    args = [ctypes.byref(exc), None, None, 64, None, None, None, None, None, None]
    assert L.sf_tune_image(ctypes.byref(d), None, 64, 64, *args) == sf.SF_EINVAL  # no pixels
    args[3] = None
    assert L.sf_tune_image(ctypes.byref(d), 64, 64, 64, *args) == sf.SF_EINVAL  # no restored buffer
