"""Discrete convolution (2.2), its DFT route (Section 2) and the sinc kernel.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings:

* (2.2) prints the index shift ``N/2 - 1``; the DFT passage below it uses
  ``(N-1)/2`` for odd ``N`` and Remark 2.1 identifies the sum with Matlab's
  ``convn(..., 'same')``.  The shift used is ``s = floor(N/2)``, which is
  ``convn``'s 'same' window for every ``N`` and equals ``(N-1)/2`` for odd
  ``N``.  Only indices inside ``[0, N)`` contribute ("legal subscripts").
* The GAF (3.1) is ``sin(pi x / Delta_x) / (pi x / Delta_x)``; for the
  workloads the bandwidth ``B = 1 / Delta_x`` is used, i.e. the kernel is
  ``sinc(B x) = sin(pi B x) / (pi B x)`` with ``sinc(0) = 1``.
* The normalisation of (7.2)/(7.3) divides by the integral over ``[-L, L]``;
  it is taken as the same midpoint sum that (2.2) uses, ``Z = dx * sum g``,
  so the discrete kernel integrates to one.  The factor is a scale only.
* Workload grids have ``N = 2**d`` samples ``x_j = j/N``; the kernel is
  sampled at ``x_m = -1/2 + m/N`` (centre ``m = N/2``) and is zero outside
  that window, so ``(2.2)`` reads ``y_j = sum_i T(j, i) f_i`` with the
  Toeplitz matrix ``T(j, i) = w_{j - i + N}`` of the length-``2N`` generator
  ``w_u = dx * g_{u - N/2}`` for ``N/2 <= u < 3N/2`` and ``0`` otherwise.
"""

from __future__ import annotations

import numpy as np


def sinc(t):
    """``sin(pi t) / (pi t)`` with value 1 at ``t = 0``."""
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    nz = t != 0
    pt = np.pi * t[nz]
    out[nz] = np.sin(pt) / pt
    return out


def sinc_kernel_samples(d: int, B: float):
    """Normalised kernel (7.2) on the workload grid: ``g_m = sinc(B x_m) / Z``.

    ``x_m = -1/2 + m/N``, ``N = 2**d``, ``Z = dx * sum_m sinc(B x_m)``.
    Returns ``(g, dx)``.
    """
    n = 1 << d
    dx = 1.0 / n
    x = -0.5 + np.arange(n, dtype=np.float64) / n
    s = sinc(B * x)
    z = dx * np.sum(s)
    return s / z, dx


def toeplitz_generator(d: int, B: float) -> np.ndarray:
    """Generator ``w`` (length ``2N``) of the convolution matrix ``T(j,i) = w_{j-i+N}``.

    ``w_u = dx * g_{u - N/2}`` for ``u`` in ``[N/2, 3N/2)``, zero elsewhere,
    with ``g`` from :func:`sinc_kernel_samples`.
    """
    n = 1 << d
    g, dx = sinc_kernel_samples(d, B)
    w = np.zeros(2 * n)
    w[n // 2: n // 2 + n] = dx * g
    return w


def conv_same(f, g, dx: float) -> np.ndarray:
    """(2.2) in 1-D by its definition: ``I_j = dx * sum_i f_i g_{j-i+s}``.

    ``s = floor(N/2)``; terms with ``j-i+s`` outside ``[0, N)`` are omitted.
    Uses numpy's direct (non-FFT) convolution sum.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = f.size
    s = n // 2
    full = np.convolve(f, g)            # full[m] = sum_i f_i g_{m-i}
    return dx * full[s: s + n]


def conv_same_fft(f, g, dx: float) -> np.ndarray:
    """(2.2) through the DFT route of Section 2 (zero padding to avoid wrap).

    Both arrays are padded with at least ``N-1`` zeros, multiplied in the
    Fourier domain, transformed back, and the window starting at ``s`` is
    taken.  Equal to :func:`conv_same` up to rounding.
    """
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = f.size
    m = 1
    while m < 2 * n - 1:
        m *= 2
    c = np.fft.irfft(np.fft.rfft(f, m) * np.fft.rfft(g, m), m)
    s = n // 2
    return dx * c[s: s + n]


def conv_same_2d(f, gy, gx, dy: float, dx: float, fft: bool = False) -> np.ndarray:
    """(2.2) with ``D = 2`` and a separable kernel ``g(x, y) = g_x(x) g_y(y)``.

    ``f`` is ``(rows, cols)``; rows are convolved with ``g_x`` (along the
    column index) and columns with ``g_y``.
    """
    op = conv_same_fft if fft else conv_same
    f = np.asarray(f, dtype=np.float64)
    t = np.stack([op(row, gx, dx) for row in f])
    return np.stack([op(col, gy, dy) for col in t.T]).T


def toeplitz_apply(f, w) -> np.ndarray:
    """``y_j = sum_i w_{j-i+N} f_i`` (exact Toeplitz product, direct sum).

    ``w`` has length ``2N``; every ``u = j - i + N`` lies in ``[1, 2N-1]``.
    """
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = f.size
    if w.size != 2 * n:
        raise ValueError("generator must have length 2N")
    full = np.convolve(f, w)            # full[m] = sum_i f_i w_{m-i}
    return full[n: 2 * n]


def toeplitz_apply_blocked(f, w, block: int = 1024, diagonals=None) -> np.ndarray:
    """The same direct sum as :func:`toeplitz_apply`, organised as the
    block-Toeplitz product ``Y_I = sum_J T_{I-J} F_J`` over blocks of ``block``
    samples (``T_delta[a, b] = w_{delta*block + a - b + N}``), one matrix
    product per block diagonal ``delta``: still ``2 N^2`` multiply-adds.

    ``diagonals`` (optional) restricts the sum to those block diagonals (a
    timing sample of the full product).
    """
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = f.size
    if w.size != 2 * n:
        raise ValueError("generator must have length 2N")
    b = min(int(block), n)
    nb = n // b
    if nb * b != n:
        raise ValueError("the block size must divide N")
    F = f.reshape(nb, b).T                      # column J holds samples J*b .. J*b + b - 1
    Y = np.zeros((b, nb))
    a = np.arange(b)
    base = a[:, None] - a[None, :] + n          # a - b' + N, in [N - b + 1, N + b - 1]
    todo = range(-(nb - 1), nb) if diagonals is None else diagonals
    for delta in todo:
        T = w[base + delta * b]                 # T_{I-J} for I - J = delta
        i0, i1 = max(0, delta), min(nb, nb + delta)
        Y[:, i0:i1] += T @ F[:, i0 - delta:i1 - delta]
    return Y.T.reshape(n)


def toeplitz_apply_fft(f, w) -> np.ndarray:
    """Same product as :func:`toeplitz_apply` through zero-padded DFTs."""
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = f.size
    m = 4 * n
    c = np.fft.irfft(np.fft.rfft(f, m) * np.fft.rfft(w, m), m)
    return c[n: 2 * n]


def toeplitz_apply_2d(f, wy, wx, fft: bool = True) -> np.ndarray:
    """Separable 2-D Toeplitz product: rows with ``wx``, then columns with ``wy``."""
    op = toeplitz_apply_fft if fft else toeplitz_apply
    f = np.asarray(f, dtype=np.float64)
    t = np.stack([op(row, wx) for row in f])
    return np.stack([op(col, wy) for col in t.T]).T


def toeplitz_dense(w) -> np.ndarray:
    """The ``N x N`` matrix ``T(j, i) = w_{j-i+N}`` built entry by entry."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size // 2
    T = np.empty((n, n))
    for j in range(n):
        for i in range(n):
            T[j, i] = w[j - i + n]
    return T


def toeplitz_transpose_apply(y, w, fft: bool = True) -> np.ndarray:
    """``x_i = sum_j w_{j-i+N} y_j`` (the adjoint of :func:`toeplitz_apply`)."""
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = y.size
    # T^T has generator w'_u = w_{2N - u}:  T^T(i, j) = w_{j-i+N} = w'_{i-j+N}
    wr = np.zeros_like(w)
    wr[1:] = w[:0:-1]
    return toeplitz_apply_fft(y, wr) if fft else toeplitz_apply(y, wr)
