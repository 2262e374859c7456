"""Seeded synthetic histogram generators (inputs only: no solver arithmetic).

Both the GPU path and the CPU oracle consume the arrays made here; this module
computes nothing of the method itself.  Every histogram is an m x n float64
array, nonnegative, summing to 1, row-major (``mu[i, j]`` is bin (i, j)), as
the paper's problem statement requires (Sec. 2.1).

The paper measures on DOTmark images (Classic, Shapes), which are not
available here; these generators stand in for them: smooth Gaussian blobs,
heavy-tailed Cauchy blobs, white noise and masked shapes with empty bins.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 240800598


def seed_for(config: int, pair: int) -> int:
    """Seed of pair ``pair`` of workload ``config``."""
    return SEED_BASE + 1000 * config + pair


def _grid(m, n):
    return np.meshgrid(np.arange(m, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")


def _normalise(h):
    h = np.asarray(h, np.float64)
    return h / h.sum()


def gaussian_blobs(m, n, nblobs, rng, floor=1e-3, sigma=(2.0, 6.0), weight=(0.5, 1.0)):
    """Sum of ``nblobs`` isotropic Gaussians (centres uniform on the grid,
    widths U[sigma], weights U[weight]) plus a constant floor, normalised."""
    ii, jj = _grid(m, n)
    h = np.zeros((m, n))
    for _ in range(nblobs):
        ci, cj = rng.uniform(0, m), rng.uniform(0, n)
        s = rng.uniform(*sigma)
        w = rng.uniform(*weight)
        h += w * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * s * s))
    return _normalise(h + floor)


def cauchy_blob(m, n, rng, scale=(5.0, 40.0), weight=(0.5, 1.0)):
    """Bivariate Cauchy density w (1 + d^2/g^2)^(-3/2), g ~ U[scale] (unnormalised)."""
    ii, jj = _grid(m, n)
    ci, cj = rng.uniform(0, m), rng.uniform(0, n)
    g = rng.uniform(*scale)
    w = rng.uniform(*weight)
    return w * (1.0 + ((ii - ci) ** 2 + (jj - cj) ** 2) / (g * g)) ** -1.5


def mixture_with_cauchy(m, n, rng, floor=1e-6):
    """1-8 Gaussian blobs plus one Cauchy blob, floor 1e-6 (large-grid recipe)."""
    nb = int(rng.integers(1, 9))
    ii, jj = _grid(m, n)
    h = np.zeros((m, n))
    for _ in range(nb):
        ci, cj = rng.uniform(0, m), rng.uniform(0, n)
        s = rng.uniform(2.0, 6.0)
        w = rng.uniform(0.5, 1.0)
        h += w * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * s * s))
    h += cauchy_blob(m, n, rng)
    return _normalise(h + floor)


def white_noise(m, n, rng):
    """U(0,1) per bin, normalised."""
    return _normalise(rng.uniform(0.0, 1.0, size=(m, n)))


def masked_shape(m, n, rng, keep=0.5):
    """Noise on a random axis-aligned ellipse; bins outside hold zero mass."""
    ii, jj = _grid(m, n)
    ci, cj = rng.uniform(0.3, 0.7) * m, rng.uniform(0.3, 0.7) * n
    ri, rj = max(1.0, keep * m / 2), max(1.0, keep * n / 2)
    mask = ((ii - ci) / ri) ** 2 + ((jj - cj) / rj) ** 2 <= 1.0
    if not mask.any():
        mask[int(ci) % m, int(cj) % n] = True
    h = rng.uniform(0.5, 1.0, size=(m, n)) * mask
    return _normalise(h)


# ---------------------------------------------------------------------------
# The five workload recipes (sizes, distributions and tolerances).
# ---------------------------------------------------------------------------

def pair_small(pair: int = 0, n: int = 32):
    """32 x 32, three Gaussian blobs + floor 1e-3 (FP64, tol 1e-6, plan)."""
    rng = np.random.default_rng(seed_for(0, pair))
    return gaussian_blobs(n, n, 3, rng), gaussian_blobs(n, n, 3, rng)


def pair_medium(kind: str = "blobs", pair: int = 0, n: int = 128):
    """128 x 128 pair: 'noise' (U(0,1)) or 'blobs' (five Gaussian blobs)."""
    rng = np.random.default_rng(seed_for(1, pair + (0 if kind == "noise" else 500)))
    if kind == "noise":
        return white_noise(n, n, rng), white_noise(n, n, rng)
    return gaussian_blobs(n, n, 5, rng), gaussian_blobs(n, n, 5, rng)


def pair_large(pair: int = 0, n: int = 512):
    """512 x 512: 1-8 Gaussian blobs + a Cauchy blob, floor 1e-6."""
    rng = np.random.default_rng(seed_for(2, pair))
    return mixture_with_cauchy(n, n, rng), mixture_with_cauchy(n, n, rng)


BATCH_SIDES = (32, 48, 64, 96, 128)


def batch_pairs(count: int = 256, sides=BATCH_SIDES):
    """``count`` pairs, side uniform in ``sides``; half 1-5 blob mixtures,
    half U(0,1) noise.  Returns a list of (mu1, mu2)."""
    out = []
    for p in range(count):
        rng = np.random.default_rng(seed_for(3, p))
        n = int(rng.choice(sides))
        if rng.uniform() < 0.5:
            out.append((gaussian_blobs(n, n, int(rng.integers(1, 6)), rng),
                        gaussian_blobs(n, n, int(rng.integers(1, 6)), rng)))
        else:
            out.append((white_noise(n, n, rng), white_noise(n, n, rng)))
    return out


SERVE_SIDES = (64, 96, 128, 192, 256)


def serving_trace(rate: float = 200.0, duration: float = 60.0, sides=SERVE_SIDES,
                  seed_pair: int = 0, max_requests: int | None = None):
    """Poisson arrivals: list of (arrival_s, n, tol, seed). Histograms are made
    lazily with ``serving_pair(n, seed)`` so a long trace stays small."""
    rng = np.random.default_rng(seed_for(4, seed_pair))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(rng.choice(sides))
        tol = 1e-4 if rng.uniform() < 0.7 else 1e-6
        out.append((t, n, tol, int(rng.integers(0, 2**31 - 1))))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out


def serving_pair(n: int, seed: int):
    rng = np.random.default_rng(seed)
    return (gaussian_blobs(n, n, int(rng.integers(1, 6)), rng),
            gaussian_blobs(n, n, int(rng.integers(1, 6)), rng))


def grid_lines(L: int, rng, spread: float = 0.7) -> np.ndarray:
    """Sorted, unevenly spaced positions of L grid lines spanning [0, L-1],
    as when lines are drawn through clustered K-means centroids (the
    non-uniform bins of the color-transfer application, Sec. 4.2): gaps are
    Gamma(spread)-distributed, so some lines bunch up and others are far
    apart."""
    if L == 1:
        return np.zeros(1)
    gaps = rng.gamma(spread, 1.0, L - 1) + 1e-3
    x = np.concatenate([[0.0], np.cumsum(gaps)])
    return x * ((L - 1) / x[-1])
