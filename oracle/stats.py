"""Plain CPU oracle of the security statistics -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; it shares no code with the GPU library.

Definitions (numpy, FP64 where floating point), for an original byte image X
and a protected byte image Y of the same planar shape (C, H, W):

* byte histograms of X and Y and the chi-square of Y against the uniform
  distribution, sum_v (h_v - N/256)^2 / (N/256) (uniformity, Sec. 6.10.1-6.10.2);
* information entropy H = -sum_v p_v log2 p_v (Eq. (3)) of X, of Y and of the
  pair (X, Y); mutual information I = H(X) + H(Y) - H(X, Y) and the normalised
  mutual information NMI = I / sqrt(H(X) H(Y)) (Sec. 6.10.5);
* block entropy (Sec. 6.10.3): Eq. (3) over the 64 samples of every 8x8 block
  (h = 8; the maximum, Eq. (4), is log2(64) = 6);
* correlation of adjacent samples (Sec. 6.6.2, Sec. 6.10.4): Pearson's r over
  every horizontally, vertically and diagonally adjacent pair of a plane (the
  report draws 10,000 or 4,096 random pairs; the full population is the limit
  of that sample), pooled over planes, population moments;
* two-dimensional correlation of X and Y (rho2, Sec. 6.10.4):
  sum (x - mx)(y - my) / sqrt(sum (x - mx)^2 sum (y - my)^2);
* Dif: percentage of differing bits between X and Y (Sec. 6.10.5; the key
  sensitivity KS of Sec. 6.10.6 is the same measure between two ciphertexts);
* PSNR = 10 log10(255^2 / MSE) (Sec. 6.10.7).

Every integer moment (sums, sums of squares and products, bit counts,
histograms) is exact; the floating-point results follow from them.
"""
from __future__ import annotations

import math

import numpy as np

from . import blocks_of, _planes

DIRS = ("h", "v", "d")


def histogram(x: np.ndarray) -> np.ndarray:
    return np.bincount(np.asarray(x, np.uint8).ravel(), minlength=256).astype(np.int64)


def entropy_bits(counts: np.ndarray) -> float:
    """Eq. (3) of a histogram (zero bins contribute nothing)."""
    c = np.asarray(counts, np.float64).ravel()
    n = c.sum()
    p = c[c > 0] / n
    return float(-(p * np.log2(p)).sum())


def chi2_uniform(counts: np.ndarray) -> float:
    c = np.asarray(counts, np.float64)
    e = c.sum() / c.size
    return float(((c - e) ** 2 / e).sum())


def joint_histogram(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """(256, 256) counts of the sample pairs (x, y)."""
    k = np.asarray(x, np.int64).ravel() * 256 + np.asarray(y, np.int64).ravel()
    return np.bincount(k, minlength=65536).reshape(256, 256)


def nmi(x: np.ndarray, y: np.ndarray):
    """(H(X), H(Y), H(X,Y), I, NMI)."""
    J = joint_histogram(x, y)
    hx, hy, hxy = entropy_bits(J.sum(1)), entropy_bits(J.sum(0)), entropy_bits(J)
    mi = hx + hy - hxy
    denom = np.sqrt(hx * hy)
    return hx, hy, hxy, mi, (mi / denom if denom > 0 else 0.0)


def block_entropy(pix: np.ndarray) -> np.ndarray:
    """(nb,) Eq. (3) over the 64 samples of each 8x8 block."""
    b = blocks_of(pix).astype(np.int64)
    nb = b.shape[0]
    cnt = np.bincount((np.arange(nb)[:, None] * 256 + b).ravel(), minlength=nb * 256).reshape(nb, 256)
    p = cnt / 64.0
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(cnt > 0, p * np.log2(np.where(cnt > 0, p, 1.0)), 0.0)
    return -t.sum(1)


def adjacent_pairs(plane: np.ndarray, d: str):
    """(first, second) samples of every adjacent pair of one plane."""
    a = np.asarray(plane, np.int64)
    if d == "h":
        return a[:, :-1], a[:, 1:]
    if d == "v":
        return a[:-1, :], a[1:, :]
    return a[:-1, :-1], a[1:, 1:]


def pair_moments(pix: np.ndarray, d: str):
    """Exact integer moments (n, Sx, Sy, Sxx, Syy, Sxy) of the adjacent pairs
    in direction d, pooled over planes."""
    pix = _planes(pix)
    m = np.zeros(6, dtype=object)
    for c in range(pix.shape[0]):
        u, v = adjacent_pairs(pix[c], d)
        m += np.array([u.size, int(u.sum()), int(v.sum()), int((u * u).sum()), int((v * v).sum()),
                       int((u * v).sum())], dtype=object)
    return tuple(int(t) for t in m)


def pearson_from_moments(n, sx, sy, sxx, syy, sxy) -> float:
    """Pearson's r from exact integer moments (population form)."""
    num = n * sxy - sx * sy                      # exact (Python integers)
    den = (n * sxx - sx * sx) * (n * syy - sy * sy)
    if den <= 0:
        return 0.0
    return float(num) / math.sqrt(float(den))


def adjacent_correlation(pix: np.ndarray, d: str) -> float:
    return pearson_from_moments(*pair_moments(pix, d))


def corr2(x: np.ndarray, y: np.ndarray) -> float:
    """Two-dimensional correlation coefficient of two images."""
    a = np.asarray(x, np.float64).ravel()
    b = np.asarray(y, np.float64).ravel()
    a = a - a.mean()
    b = b - b.mean()
    den = np.sqrt((a * a).sum() * (b * b).sum())
    return float((a * b).sum() / den) if den > 0 else 0.0


def bit_difference_percent(x: np.ndarray, y: np.ndarray) -> float:
    d = np.bitwise_xor(np.asarray(x, np.uint8).ravel(), np.asarray(y, np.uint8).ravel())
    return 100.0 * float(np.unpackbits(d).sum()) / (8.0 * d.size)


def psnr(x: np.ndarray, y: np.ndarray) -> float:
    e = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    mse = float((e * e).mean())
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def expected_block_entropy_uniform(n: int = 64, k: int = 256) -> float:
    """E[H] of n independent samples uniform over k symbols, in closed form:
    by linearity, k * sum_c P(count = c) * (-(c/n) log2(c/n)), count ~ Binomial(n, 1/k)."""
    from math import comb, log2
    p = 1.0 / k
    return k * sum(comb(n, c) * p ** c * (1 - p) ** (n - c) * (-(c / n) * log2(c / n)) for c in range(1, n + 1))


def security_stats(x: np.ndarray, y: np.ndarray) -> dict:
    """All statistics of the pair (original x, protected y)."""
    x = _planes(x)
    y = _planes(y)
    assert x.shape == y.shape
    hx, hy, hxy, mi, n_mi = nmi(x, y)
    bx, by = block_entropy(x), block_entropy(y)
    out = {
        "samples": x.size,
        "hist_x": histogram(x), "hist_y": histogram(y), "chi2_y": chi2_uniform(histogram(y)),
        "entropy_x": hx, "entropy_y": hy, "joint_entropy": hxy, "mutual_information": mi, "nmi": n_mi,
        "block_entropy_x": bx, "block_entropy_y": by,
        "corr2": corr2(x, y), "dif": bit_difference_percent(x, y), "psnr": psnr(x, y),
    }
    for d in DIRS:
        out["moments_x_" + d] = pair_moments(x, d)
        out["moments_y_" + d] = pair_moments(y, d)
        out["corr_x_" + d] = pearson_from_moments(*out["moments_x_" + d])
        out["corr_y_" + d] = pearson_from_moments(*out["moments_y_" + d])
    return out


__all__ = ["histogram", "entropy_bits", "chi2_uniform", "joint_histogram", "nmi", "block_entropy",
           "adjacent_pairs", "pair_moments", "pearson_from_moments", "adjacent_correlation", "corr2",
           "bit_difference_percent", "psnr", "expected_block_entropy_uniform", "security_stats", "DIRS"]
