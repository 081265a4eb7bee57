"""Seeded generators for the synthetic SAR-like workloads and the paper's examples.

All generators use ``numpy.random.default_rng(seed)`` and draw in the order
written in each docstring.  They return float64 arrays; callers cast to the
working precision.  Nothing here depends on the QTT method.

Grids
-----
* Workloads (range lines, images): ``N = 2**d`` samples at ``x_j = j / N`` on
  ``[0, 1)``.  Images are ``(rows, cols)`` row-major with ``y = r / N_y``,
  ``x = c / N_x``.
* Paper examples (Section 7): odd ``N = 2**(K-1) - 1`` midpoint samples
  ``x_j = -L + dx/2 + j dx`` with ``dx = 2L/N`` (Section 2 grid), noise
  ``N(0, s)`` read with ``s`` the standard deviation.
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# 1-D range lines
# ---------------------------------------------------------------------------

def gaussian_bumps_1d(d: int, seed: int = 1, n_bumps: int = 5, width: float = 2e-3,
                      noise_rel: float = 0.05):
    """Sum of Gaussian bumps plus white noise (1-D plain-method workload).

    Draw order: centres ``c ~ U(0,1)^n``, amplitudes ``a ~ U(0.5,1)^n``,
    noise ``xi ~ N(0,1)^N``.  ``width`` is the Gaussian standard deviation.
    The noise is scaled to ``noise_rel * max|s|``.

    Returns ``(noisy, clean)``.
    """
    n = 1 << d
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, n_bumps)
    a = rng.uniform(0.5, 1.0, n_bumps)
    x = np.arange(n, dtype=np.float64) / n
    s = np.zeros(n)
    for ci, ai in zip(c, a):
        s += ai * np.exp(-((x - ci) ** 2) / (2.0 * width * width))
    xi = rng.standard_normal(n)
    noisy = s + noise_rel * np.max(np.abs(s)) * xi
    return noisy, s


def scatterers_1d(d: int, seed: int = 2, n_scatterers: int = 64,
                  amp_lo: float = 0.1, noise_rel: float = 0.05,
                  window_samples: float = 8.0, background: float = 0.2):
    """Gaussian-windowed point scatterers on a cosine background plus noise.

    Draw order: positions ``U(0,1)^n``, amplitudes ``U(amp_lo,1)^n``,
    background wavenumber ``k ~ integers{1..4}``, noise ``N(0,1)^N``.  Each
    scatterer is ``amp * exp(-(x-pos)^2 / (2 (window_samples/N)^2))``; the
    background is ``background * cos(2 pi k x)``; the noise is scaled to
    ``noise_rel * max|clean|``.

    Returns ``(noisy, clean)``.
    """
    n = 1 << d
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, n_scatterers)
    amp = rng.uniform(amp_lo, 1.0, n_scatterers)
    k = int(rng.integers(1, 5))
    x = np.arange(n, dtype=np.float64) / n
    s = background * np.cos(2.0 * np.pi * k * x)
    w = window_samples / n
    # each window is negligible beyond ~12 std; evaluate locally for speed
    half = int(np.ceil(12.0 * window_samples)) + 1
    for p, a in zip(pos, amp):
        c = int(round(p * n))
        lo, hi = max(0, c - half), min(n, c + half + 1)
        xs = x[lo:hi]
        s[lo:hi] += a * np.exp(-((xs - p) ** 2) / (2.0 * w * w))
    xi = rng.standard_normal(n)
    noisy = s + noise_rel * np.max(np.abs(s)) * xi
    return noisy, s


def sar_image_2d(dy: int = 12, dx: int = 12, seed: int = 3, n_scatterers: int = 200,
                 snr_db: float = 10.0, background: float = 0.2):
    """SAR-like image: single-pixel scatterers on a smooth background + noise.

    Draw order: ``(kx, ky) ~ integers{1..4}^2``, scatterer rows, columns
    ``integers[0,N)^n`` each, amplitudes ``U(0.2,1)^n``, noise ``N(0,1)``
    image.  Background ``background*cos(2 pi kx x) cos(2 pi ky y)``; the
    noise standard deviation is ``rms(clean) / 10**(snr_db/20)``.

    Returns ``(noisy, clean)`` of shape ``(2**dy, 2**dx)`` (row-major).
    """
    ny, nx = 1 << dy, 1 << dx
    rng = np.random.default_rng(seed)
    kx, ky = (int(v) for v in rng.integers(1, 5, size=2))
    rows = rng.integers(0, ny, n_scatterers)
    cols = rng.integers(0, nx, n_scatterers)
    amp = rng.uniform(0.2, 1.0, n_scatterers)
    y = np.arange(ny, dtype=np.float64) / ny
    x = np.arange(nx, dtype=np.float64) / nx
    s = background * np.outer(np.cos(2.0 * np.pi * ky * y), np.cos(2.0 * np.pi * kx * x))
    np.add.at(s, (rows, cols), amp)
    sigma = np.sqrt(np.mean(s * s)) / (10.0 ** (snr_db / 20.0))
    noisy = s + sigma * rng.standard_normal((ny, nx))
    return noisy, s


def batch_lines(n_lines: int = 4096, d_lo: int = 10, d_hi: int = 16, seed: int = 4,
                b_lo: float = 100.0, b_hi: float = 2000.0, lines=None):
    """Batch of independent range lines of uneven length.

    The master generator (``seed``) draws ``d_l ~ integers{d_lo..d_hi}`` for
    every line.  Line ``l`` then uses its own generator seeded
    ``seed*1_000_000 + l`` and draws: scatterer count ``integers{8..32}``,
    then the :func:`scatterers_1d` draws (positions, amplitudes, background
    wavenumber, noise), then its kernel bandwidth ``B_l ~ U(b_lo, b_hi)``.

    ``lines`` optionally restricts which line indices are generated (the
    per-line values do not depend on which others are generated).

    Returns ``(ds, Bs, noisy_list, clean_list)`` for the generated lines.
    """
    master = np.random.default_rng(seed)
    ds_all = master.integers(d_lo, d_hi + 1, n_lines)
    idx = range(n_lines) if lines is None else lines
    ds, bs, noisy_l, clean_l = [], [], [], []
    for li in idx:
        rng = np.random.default_rng(seed * 1_000_000 + int(li))
        d = int(ds_all[li])
        n = 1 << d
        nsc = int(rng.integers(8, 33))
        pos = rng.uniform(0.0, 1.0, nsc)
        amp = rng.uniform(0.1, 1.0, nsc)
        k = int(rng.integers(1, 5))
        x = np.arange(n, dtype=np.float64) / n
        s = 0.2 * np.cos(2.0 * np.pi * k * x)
        w = 8.0 / n
        for p, a in zip(pos, amp):
            s += a * np.exp(-((x - p) ** 2) / (2.0 * w * w))
        xi = rng.standard_normal(n)
        noisy = s + 0.05 * np.max(np.abs(s)) * xi
        b = float(rng.uniform(b_lo, b_hi))
        ds.append(d)
        bs.append(b)
        noisy_l.append(noisy)
        clean_l.append(s)
    return ds, bs, noisy_l, clean_l


def diff_workload(d: int = 22, seed: int = 5):
    """Differentiation workload: the Gaussian-bump generator at size ``2**d``.

    Returns ``(noisy, clean)``; the target, bandwidths and starting point are
    set by the caller (target bandwidth 200, initial bandwidth 220).
    """
    return gaussian_bumps_1d(d, seed=seed)


WORKLOADS = {
    "line_d12": dict(gen="gaussian_bumps_1d", d=12, seed=1, B=200.0, eps=1e-3, max_rank=0),
    "line_d20": dict(gen="scatterers_1d", d=20, seed=2, B=2000.0, eps=1e-4, max_rank=32),
    "image_4096": dict(gen="sar_image_2d", dy=12, dx=12, seed=3, B=1000.0, eps=1e-3, max_rank=32),
    "batch_4096": dict(gen="batch_lines", n_lines=4096, seed=4, eps=1e-4, max_rank=32),
    "diff_d22": dict(gen="diff_workload", d=22, seed=5, B_true=200.0, B0=220.0, eps=1e-4,
                     max_rank=32),
}


# ---------------------------------------------------------------------------
# The paper's analytic examples (Section 7)
# ---------------------------------------------------------------------------

def _midpoint_grid(K: int, L: float, full_grid: bool = False):
    n = (1 << K) if full_grid else (1 << (K - 1)) - 1
    dx = 2.0 * L / n
    x = -L + dx / 2.0 + dx * np.arange(n, dtype=np.float64)
    return x, dx


def paper_example1(K: int, seed: int = 0, full_grid: bool = False):
    """Example 1: smooth damped oscillation on [-10,10], noise std 0.02.

    Returns ``(noisy, clean, x, dx)`` with ``N = 2**(K-1) - 1`` samples
    (``N = 2**K`` with ``full_grid``).
    """
    x, dx = _midpoint_grid(K, 10.0, full_grid)
    f = np.exp(-(3.0 * x / 10.0) ** 2) * (0.4 * np.sin(8 * np.pi * x) - 0.7 * np.cos(6 * np.pi * x))
    rng = np.random.default_rng(seed)
    return f + 0.02 * rng.standard_normal(x.size), f, x, dx


def paper_example2(K: int, seed: int = 0):
    """Example 2: highly oscillatory signal on [-1,1], noise std 0.01.

    Returns ``(noisy, clean, x, dx)``.
    """
    x, dx = _midpoint_grid(K, 1.0)
    f = np.exp(-(3.0 * x) ** 2) * (0.9 * np.sin(2 * x * np.pi / (5 * dx))
                                   + 1.4 * np.cos(x * np.pi / (3 * dx)))
    rng = np.random.default_rng(seed)
    return f + 0.01 * rng.standard_normal(x.size), f, x, dx


def paper_example3(K: int, seed: int = 0):
    """Example 3: 2-D damped oscillation on [-1,1]^2, noise std 0.1.

    ``f[j, k] = f(x_j, y_k)``; returns ``(noisy, clean, x, dx)``.
    """
    x, dx = _midpoint_grid(K, 1.0)
    X, Y = np.meshgrid(x, x, indexing="ij")
    f = np.exp(-((2 * X) ** 2 + (2 * Y) ** 2)) * (np.sin(2 * np.pi * X) - np.cos(7 * np.pi * Y)
                                                 + np.cos(4 * np.pi * X * Y)
                                                 - np.sin(3 * np.pi * X * Y))
    rng = np.random.default_rng(seed)
    return f + 0.1 * rng.standard_normal(f.shape), f, x, dx


def closed_form_signal(kind: str, d: int, param: float = 1.0):
    """Analytic signals with known QTT ranks on ``x_j = j / 2**d``.

    ``kind``: ``"exp"`` (``exp(param*x)``), ``"sin"``/``"cos"``
    (``sin(2 pi param x + 0.3)``), ``"poly"`` (degree ``int(param)``
    polynomial with fixed non-zero coefficients), ``"zero"``.
    """
    n = 1 << d
    x = np.arange(n, dtype=np.float64) / n
    if kind == "exp":
        return np.exp(param * x)
    if kind == "sin":
        return np.sin(2 * np.pi * param * x + 0.3)
    if kind == "cos":
        return np.cos(2 * np.pi * param * x + 0.3)
    if kind == "poly":
        p = int(param)
        coef = [(-1.0) ** c * (1.0 + 0.5 * c) for c in range(p + 1)]
        return sum(cc * (x - 0.37) ** c for c, cc in enumerate(coef))
    if kind == "zero":
        return np.zeros(n)
    raise ValueError(kind)
