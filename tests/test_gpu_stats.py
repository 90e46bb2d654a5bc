"""GPU parity of the security statistics against the oracle, through the C
ABI.  Integer results (histograms, the joint histogram, pair and cross
moments, differing bits) must be identical; FP64 results within 1e-12
(entropies, chi-square, correlations, PSNR: each is a few FP64 operations on
exact integers, or sums of 256 / 65536 such terms), block entropies within
float32 rounding of the stored value (2^-21 for values up to 6)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import pixel as opx
from oracle import stats as ost

sf = pytest.importorskip("paper_1512_02951_amd")
from paper_1512_02951_amd import pixel, stats  # noqa: E402

pytestmark = pytest.mark.gpu


def _close(a, b, tol=1e-12):
    if math.isinf(b):
        return math.isinf(a)
    return abs(a - b) <= tol * max(1.0, abs(b))


def _compare(x, y, label, full_blocks=True):
    print("case:", label, x.shape, flush=True)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    r = stats.StatsRunner(xd.device)
    C, H, W = x.shape
    be = torch.empty(2 * C * (H // 8) * (W // 8), dtype=torch.float32, device="cuda")
    r.launch(xd, yd, be)
    got = r.result()
    J = r.joint_histogram().cpu().numpy()
    ref = ost.security_stats(x, y)
    assert got["samples"] == ref["samples"]
    assert got["hist_x"] == ref["hist_x"].tolist() and got["hist_y"] == ref["hist_y"].tolist()
    assert np.array_equal(J, ost.joint_histogram(x, y))
    for im in ("x", "y"):
        for d in ost.DIRS:
            k = "moments_%s_%s" % (im, d)
            assert got[k] == ref[k], k
            assert _close(got["corr_%s_%s" % (im, d)], ref["corr_%s_%s" % (im, d)]), (im, d)
    xs, ys = x.astype(np.int64), y.astype(np.int64)
    assert got["cross"] == (x.size, int(xs.sum()), int(ys.sum()), int((xs * xs).sum()), int((ys * ys).sum()),
                            int((xs * ys).sum()))
    assert got["bits_differing"] == int(np.unpackbits(np.bitwise_xor(x, y).ravel()).sum())
    for k in ("chi2_y", "entropy_x", "entropy_y", "joint_entropy", "mutual_information", "corr2", "dif", "psnr"):
        assert _close(got[k], ref[k]), (k, got[k], ref[k])
    assert _close(got["nmi"], ref["nmi"], 1e-10)
    b = be.cpu().numpy()
    nb = C * (H // 8) * (W // 8)
    for im, bref in (("x", ref["block_entropy_x"]), ("y", ref["block_entropy_y"])):
        gb = b[:nb] if im == "x" else b[nb:]
        assert np.abs(gb - bref).max() <= 2.0 ** -21, im
        st = got["block_entropy_" + im]
        assert _close(st[0], bref.mean(), 1e-12) and abs(st[1] - bref.std()) <= 1e-9
        assert _close(st[2], bref.min()) and _close(st[3], bref.max())
    return got


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 24, 40), (1, 72, 136), (2, 64, 264), (1, 16, 1032), (1, 8, 4104)])
def test_against_strong_public_fragment(shape):
    C, H, W = shape
    x = synth.image(H, W, C, 2, 8).numpy()
    y = opx.frag(x, oracle.prefix_mask(5), strong=True)["public"]
    _compare(x, y, "strong public")


def test_degenerate_and_limit_cases():
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, (2, 32, 72)).astype(np.uint8)
    g = _compare(x, x.copy(), "identical")
    assert g["dif"] == 0.0 and math.isinf(g["psnr"]) and abs(g["nmi"] - 1) < 1e-12
    g = _compare(x, (255 - x).astype(np.uint8), "complement")
    assert g["dif"] == 100.0 and abs(g["corr2"] + 1) < 1e-12
    c = np.full((1, 16, 16), 77, np.uint8)
    g = _compare(c, c.copy(), "constant")
    assert g["nmi"] == 0.0 and g["corr_x_h"] == 0.0 and g["block_entropy_x"][0] == 0.0
    ramp = np.tile(np.arange(256, dtype=np.uint8), (16, 1))[None]
    g = _compare(ramp, rng.integers(0, 256, ramp.shape).astype(np.uint8), "ramp")
    assert abs(g["corr_x_h"] - 1) < 1e-12


def test_full_size_4096_rgb_strong_public():
    H = W = 4096
    C = 3
    mask = sf.prefix_mask(5)
    key, c0 = synth.aes_key(2), synth.ctr0(2, 0)
    x = synth.image(H, W, C, 2, 0, device="cuda")
    y = pixel.pixel_frag_image(x, mask, True, key, c0).public
    r = stats.StatsRunner(x.device)
    r.launch(x, y)
    got = r.result()
    xn, yn = x.cpu().numpy(), y.cpu().numpy()
    assert got["hist_y"] == ost.histogram(yn).tolist()
    assert np.array_equal(r.joint_histogram().cpu().numpy(), ost.joint_histogram(xn, yn))
    for d in ost.DIRS:
        assert got["moments_x_" + d] == ost.pair_moments(xn, d)
        assert got["moments_y_" + d] == ost.pair_moments(yn, d)
    hx, hy, hxy, mi, nmi = ost.nmi(xn, yn)
    assert _close(got["nmi"], nmi, 1e-10) and _close(got["joint_entropy"], hxy)
    assert _close(got["corr2"], ost.corr2(xn, yn)) and _close(got["psnr"], ost.psnr(xn, yn))
    # the report's qualitative claims for the strong level (Sec. 6.6, 6.10)
    assert abs(got["corr_y_h"]) < 0.01 and got["corr_x_h"] > 0.5
    assert got["chi2_y"] < 255 + 10 * math.sqrt(510)
    assert abs(got["block_entropy_y"][0] - ost.expected_block_entropy_uniform()) < 0.01


def test_tall_narrow_image_sums_stay_exact():
    # W = 8: one lane pair per band, 2^24 bands (4096 per wave): far more than
    # a 32-bit lane sum of squares could hold without the periodic flush.
    # Constant images give every moment in closed form.
    C, H, W = 1, 1 << 27, 8
    x = torch.full((C, H, W), 255, dtype=torch.uint8, device="cuda")
    y = torch.full((C, H, W), 254, dtype=torch.uint8, device="cuda")
    r = stats.StatsRunner(x.device)
    r.launch(x, y)
    g = r.result()
    N = C * H * W
    n = {"h": H * (W - 1), "v": (H - 1) * W, "d": (H - 1) * (W - 1)}
    for d in ost.DIRS:
        assert g["moments_x_" + d] == (n[d], 255 * n[d], 255 * n[d], 65025 * n[d], 65025 * n[d], 65025 * n[d])
        assert g["moments_y_" + d] == (n[d], 254 * n[d], 254 * n[d], 64516 * n[d], 64516 * n[d], 64516 * n[d])
    assert g["cross"] == (N, 255 * N, 254 * N, 65025 * N, 64516 * N, 255 * 254 * N)
    assert g["bits_differing"] == N                      # 255 ^ 254 = 1: one bit per sample
    assert g["hist_x"][255] == N and g["hist_y"][254] == N
    assert max(abs(v) for v in g["block_entropy_x"]) < 1e-12
    assert abs(g["psnr"] - 10 * math.log10(255 ** 2)) < 1e-12


def test_errors():
    x = torch.zeros((1, 12, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SefragError) as e:
        stats.security_stats(x, x)
    assert e.value.code == sf.SF_ESHAPE
