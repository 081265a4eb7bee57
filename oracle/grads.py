"""Gradients of the convolution + reconstruction loss, by plain definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss is ``L(F, B) = || T(w(B)) full(F) - t ||^2`` where ``full(F)`` is
the QTT vector of the signal cores (Algorithm 3), ``T(w)`` the Toeplitz form
of the discrete convolution (2.2) with generator ``w`` and ``w(B)`` the
normalised sinc generator of bandwidth ``B`` (kernel (7.2), GAF (3.1)).
The paper gives no derivative; these are written from the chain rule:

* ``dL/dy = 2 (y - t)``;
* ``dL/df = T^T dL/dy`` (a correlation);
* ``dL/dG_k[a, i, b] = sum_{j : j_k = i} (dL/df)_j  L_{<k}(j)[a]  R_{>k}(j)[b]``
  where ``L_{<k}(j)`` and ``R_{>k}(j)`` are the products of the core slices
  before and after mode ``k`` (computed here from the full left and right
  interface matrices);
* ``dL/dw_u = sum_{j - i + N = u} (dL/dy)_j f_i``;
* ``dL/dB = sum_u dL/dw_u dw_u/dB`` with ``w_u = s_m / S``,
  ``s_m = sinc(B x_m)``, ``S = sum_m s_m`` (the ``dx`` of (2.2) cancels the
  normalisation), so ``dw_u/dB = s'_m / S - s_m (sum s') / S^2`` and
  ``s' = d sinc(B x)/dB = (cos(pi B x) - sinc(B x)) / B`` (0 at ``x = 0``).
"""

from __future__ import annotations

import numpy as np

from . import conv, tt


def sinc_dB(d: int, B: float):
    """``(s, ds/dB)`` of ``s_m = sinc(B x_m)`` on the workload kernel grid."""
    n = 1 << d
    x = -0.5 + np.arange(n, dtype=np.float64) / n
    s = conv.sinc(B * x)
    ds = np.where(x == 0.0, 0.0, (np.cos(np.pi * B * x) - s) / B)
    return s, ds


def generator_dB(d: int, B: float) -> np.ndarray:
    """``dw/dB`` of the normalised generator (length ``2N``)."""
    n = 1 << d
    s, ds = sinc_dB(d, B)
    S = np.sum(s)
    dg = ds / S - s * np.sum(ds) / (S * S)
    out = np.zeros(2 * n)
    out[n // 2: n // 2 + n] = dg
    return out


def loss(cores, B: float, target, w=None) -> float:
    """``L = ||T(w) full(F) - t||^2``; ``w`` defaults to the exact generator ``w(B)``."""
    f = tt.tt_full(cores)
    d = tt.log2_exact(f.size)
    if w is None:
        w = conv.toeplitz_generator(d, B)
    y = conv.toeplitz_apply_fft(f, w)
    r = y - np.asarray(target, dtype=np.float64)
    return float(r @ r)


def _left_interfaces(cores):
    """``Lf[k]``: matrix ``2**k x r_k`` of products of the first ``k`` cores."""
    out = [np.ones((1, 1))]
    A = np.ones((1, 1))
    for G in cores[:-1]:
        r0, _, r1 = G.shape
        # rows: position index with the new bit as the most significant one
        A = np.concatenate([A @ G[:, 0, :], A @ G[:, 1, :]], axis=0)
        out.append(A)
    return out


def _right_interfaces(cores):
    """``Rf[k]``: matrix ``r_k x 2**(K-k)`` of products of cores ``k+1..K``."""
    K = len(cores)
    out = [None] * (K + 1)
    B = np.ones((1, 1))
    out[K] = B
    for k in range(K - 1, 0, -1):
        G = cores[k]
        # columns: position index of bits k+1..K, bit k+1 least significant
        Bn = np.empty((G.shape[0], 2 * B.shape[1]))
        Bn[:, 0::2] = G[:, 0, :] @ B
        Bn[:, 1::2] = G[:, 1, :] @ B
        B = Bn
        out[k] = B
    return out


def grads(cores, B: float, target, w=None, dw=None):
    """Return ``(L, [dL/dG_k], dL/dB, dL/dw, dL/df)`` by full-format contractions.

    ``w`` (generator) and ``dw`` (its derivative in ``B``) default to the
    exact ones; passing approximations (e.g. the full arrays of their QTTs)
    gives the gradients of the loss with those in place, at fixed ranks.
    """
    f = tt.tt_full(cores)
    n = f.size
    d = tt.log2_exact(n)
    if w is None:
        w = conv.toeplitz_generator(d, B)
    if dw is None:
        dw = generator_dB(d, B)
    y = conv.toeplitz_apply_fft(f, w)
    r = y - np.asarray(target, dtype=np.float64)
    L = float(r @ r)
    gy = 2.0 * r
    gf = conv.toeplitz_transpose_apply(gy, w)
    # dL/dw_u = sum_j gy_j f_{j + N - u}: a correlation of gy with f
    m = 4 * n
    c = np.fft.irfft(np.fft.rfft(gy, m) * np.conj(np.fft.rfft(f, m)), m)
    # c[s] = sum_j gy_j f_{j - s} (no wrap-around for |s| < N); u = j - i + N = N + s
    gw = np.zeros(2 * n)
    u = np.arange(1, 2 * n)
    gw[1:] = c[(u - n) % m]
    gB = float(gw @ dw)
    gcores = full_adjoint(cores, gf)
    return L, gcores, gB, gw, gf


def full_adjoint(cores, g):
    """``[d<g, full(F)>/dG_k]``: ``g`` contracted with the left and right
    interfaces of every core (the products of the slices before and after it)."""
    g = np.asarray(g, dtype=np.float64)
    Lf = _left_interfaces(cores)
    Rf = _right_interfaces(cores)
    gcores = []
    for k, G in enumerate(cores):
        Lk = Lf[k]                # 2**k x r_{k}   (bits 1..k)
        Rk = Rf[k + 1]            # r_{k+1} x 2**(K-k-1) (bits k+2..K)
        out = np.zeros_like(G)
        # position j = low + 2**k * i + 2**(k+1) * high
        g3 = g.reshape((Rk.shape[1], 2, Lk.shape[0]))   # [high, i, low] (C order: low fastest)
        for i in range(2):
            M = g3[:, i, :]                                 # high x low
            out[:, i, :] = Lk.T @ M.T @ Rk.T
        gcores.append(out)
    return gcores
