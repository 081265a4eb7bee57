"""Pins of the oracle's convolution (2.2), DFT route (Section 2) and sinc kernel."""

import json
import os

import numpy as np
import pytest

from oracle import conv, pipeline
from synthetic import generators as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _brute_same(f, g, dx):
    n = f.size
    s = n // 2
    out = np.zeros(n)
    for j in range(n):
        acc = 0.0
        for i in range(n):
            m = j - i + s
            if 0 <= m < n:
                acc += f[i] * g[m]
        out[j] = dx * acc
    return out


@pytest.mark.parametrize("n", [1, 2, 7, 16, 33, 256])
def test_conv_same_bruteforce(n):
    rng = np.random.default_rng(n)
    f, g = rng.standard_normal(n), rng.standard_normal(n)
    ref = _brute_same(f, g, 0.25)
    assert np.allclose(conv.conv_same(f, g, 0.25), ref, rtol=0, atol=1e-12)
    assert np.allclose(conv.conv_same_fft(f, g, 0.25), ref, rtol=0, atol=1e-12)


def test_conv_same_matches_matlab_same_window_odd():
    # for odd N the shift is (N-1)/2 as in the DFT passage of Section 2
    n = 9
    f = np.zeros(n)
    f[0] = 1.0
    g = np.arange(1.0, n + 1)
    out = conv.conv_same(f, g, 1.0)
    assert np.array_equal(out, np.concatenate([g[4:], np.zeros(4)]))


@pytest.mark.parametrize("d", [1, 3, 6, 8])
def test_toeplitz_apply_vs_dense(d):
    rng = np.random.default_rng(d)
    n = 1 << d
    w = rng.standard_normal(2 * n)
    f = rng.standard_normal(n)
    T = conv.toeplitz_dense(w)
    assert np.allclose(conv.toeplitz_apply(f, w), T @ f, atol=1e-12)
    assert np.allclose(conv.toeplitz_apply_fft(f, w), T @ f, atol=1e-11)
    y = rng.standard_normal(n)
    assert np.allclose(conv.toeplitz_transpose_apply(y, w), T.T @ y, atol=1e-11)
    assert np.allclose(conv.toeplitz_transpose_apply(y, w, fft=False), T.T @ y, atol=1e-12)


@pytest.mark.parametrize("d,B", [(6, 10.0), (10, 200.0), (12, 200.0)])
def test_generator_form_equals_2_2(d, B):
    f = G.gaussian_bumps_1d(d, seed=d)[0]
    g, dx = conv.sinc_kernel_samples(d, B)
    a = conv.conv_same(f, g, dx)
    b = conv.toeplitz_apply(f, conv.toeplitz_generator(d, B))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_gaussian_convolution_second_order():
    """(2.2) against the exact Gaussian*Gaussian convolution (midpoint-rule sum)."""
    errs = []
    for d in (7, 8, 9):
        n = 1 << d
        L = 6.0
        dx = 2 * L / n
        x = -L + dx / 2 + dx * np.arange(n)
        a, b = 0.5, 0.7
        f = np.exp(-x * x / (2 * a * a))
        g = np.exp(-x * x / (2 * b * b))
        out = conv.conv_same(f, g, dx)
        # exact: (f*g)(x) = sqrt(2 pi) a b / sqrt(a^2+b^2) exp(-x^2 / (2(a^2+b^2)))
        # the 'same' window of an even N is offset by dx/2 relative to x
        xs = x + dx / 2.0
        exact = np.sqrt(2 * np.pi) * a * b / np.hypot(a, b) * np.exp(-xs * xs / (2 * (a * a + b * b)))
        errs.append(np.max(np.abs(out - exact)))
    # spectral accuracy for smooth decaying integrands makes the error tiny
    assert max(errs) < 1e-12


def test_sinc_kernel_properties():
    d, B = 12, 200.0
    g, dx = conv.sinc_kernel_samples(d, B)
    n = 1 << d
    assert np.argmax(g) == n // 2                           # centre at x = 0
    assert dx * np.sum(g) == pytest.approx(1.0, rel=1e-14)  # normalised
    # first zero of sin(pi B x)/(pi B x) at x = 1/B (resolution, Section 3)
    x = -0.5 + np.arange(n) / n
    k = n // 2 + int(round(n / B))
    if abs(x[k] - 1.0 / B) < 1e-15:
        assert abs(g[k]) < 1e-12 * g[n // 2]
    assert conv.sinc(np.array([0.0]))[0] == 1.0
    assert conv.sinc(np.array([1.0]))[0] == pytest.approx(0.0, abs=1e-16)
    assert conv.sinc(np.array([0.5]))[0] == pytest.approx(2 / np.pi)


def test_sinc_first_zero_on_grid():
    d = 10
    n = 1 << d
    B = n / 8.0                                            # 1/B is exactly 8 samples
    g, _ = conv.sinc_kernel_samples(d, B)
    assert abs(g[n // 2 + 8]) < 1e-15 * g[n // 2]
    assert abs(g[n // 2 - 8]) < 1e-15 * g[n // 2]
    assert g[n // 2 + 7] > 0 and g[n // 2 + 9] < 0


def test_table_7_1_noisy_convolution_error():
    gold = json.load(open(os.path.join(GOLD, "table_7_1_noisy_conv_error.json")))["values"]

    def kern(x, res, dx):
        g = conv.sinc(x / res)
        return g / (dx * g.sum())

    got = {"example1": [], "example2": [], "example3": []}
    for seed in range(3):
        for name, gen, fac in (("example1", G.paper_example1, 4), ("example2", G.paper_example2, 2)):
            xn, f, x, dx = gen(20, seed)
            g = kern(x, fac * dx, dx)
            got[name].append(pipeline.relative_error(conv.conv_same_fft(xn, g, dx),
                                                     conv.conv_same_fft(f, g, dx)))
        xn, f, x, dx = G.paper_example3(10, seed)
        g = kern(x, 2 * dx, dx)
        got["example3"].append(pipeline.relative_error(conv.conv_same_2d(xn, g, g, dx, dx),
                                                       conv.conv_same_2d(f, g, g, dx, dx)))
    for k, v in gold.items():
        assert np.mean(got[k]) == pytest.approx(v, rel=0.05), (k, got[k])


def test_table_7_1_rejects_variance_reading():
    """Reading N(0, s) with s as the variance misses the printed column by far."""
    xn, f, x, dx = G.paper_example1(16, 0)
    noise = (xn - f) / 0.02 * np.sqrt(0.02)
    g = conv.sinc(x / (4 * dx))
    g /= dx * g.sum()
    e_std = pipeline.relative_error(conv.conv_same_fft(xn, g, dx), conv.conv_same_fft(f, g, dx))
    e_var = pipeline.relative_error(conv.conv_same_fft(f + noise, g, dx), conv.conv_same_fft(f, g, dx))
    assert e_var > 4 * e_std


@pytest.mark.parametrize("d,block", [(4, 1), (6, 8), (9, 64), (10, 1024)])
def test_blocked_toeplitz_equals_direct_sum(d, block):
    """The block-Toeplitz organisation of (2.2) gives the direct sum."""
    rng = np.random.default_rng(d)
    n = 1 << d
    f = rng.standard_normal(n)
    w = rng.standard_normal(2 * n)
    want = conv.toeplitz_apply(f, w)
    got = conv.toeplitz_apply_blocked(f, w, block=block)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # the block diagonals partition the sum
    nb = n // min(block, n)
    half = conv.toeplitz_apply_blocked(f, w, block=block, diagonals=range(-(nb - 1), 1))
    rest = conv.toeplitz_apply_blocked(f, w, block=block, diagonals=range(1, nb))
    assert np.allclose(half + rest, want, rtol=0, atol=1e-12 * np.abs(want).max())
