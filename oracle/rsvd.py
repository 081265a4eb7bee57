"""Randomized range finder and RSVD (Algorithms 4 and 5 of Appendix A) and the
TT-SVD sweep that takes every truncated SVD from them, in float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Gaussian test matrix is bit-defined so that an independent GPU
implementation draws the same one: entry ``Omega[row, col]`` of sweep step
``step`` comes from one call of the counter-based generator Philox-4x32-10
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
3", SC 2011) with counter ``(row, col, step, 0)`` and key ``(seed mod 2^32,
seed >> 32)``; its first two output words ``x0, x1`` give the uniforms
``u = (x + 1/2) 2^-32`` in (0, 1) and the Box-Muller transform
``sqrt(-2 ln u1) cos(2 pi u2)`` gives one standard normal.

Readings: Algorithm 4 is applied to the unfolding ``A`` (``m x n``) of each
step with ``ell = k + p`` columns.  With ``ell >= m`` the sketch ``Y``
(``m x ell``, full row rank with probability one) spans all of ``R^m``, so
``Q`` is an orthogonal ``m x m`` basis, ``B = Q^T A`` has the singular values
of ``A`` and ``U = Q U~`` its left singular vectors: the step is the exact
truncated SVD, and the sweep takes it directly without drawing ``Omega``.
The rank of each step is then chosen from the singular values of
``B = Q^T A`` by the rule of Algorithm 1 (tolerance and cap), as in the plain
sweep.  ``Y = A Omega`` is accumulated over blocks of columns of ``A`` (rows
of ``Omega``), so the test matrix is never held whole.
"""

from __future__ import annotations

import math

import numpy as np

from . import tt

_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox-4x32 with 10 rounds on uint64 numpy arrays holding 32-bit words.

    ``ctr`` is a sequence of 4 arrays (or ints), ``key`` of 2; returns the 4
    output words.  Each round multiplies words 0 and 2 by the two constants,
    mixes the high halves with the other words and the key, and the key is
    advanced by the two Weyl constants between rounds.
    """
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = c[0] * np.uint64(_M0)
        p1 = c[2] * np.uint64(_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def gaussian_matrix(nrows: int, ncols: int, step: int, seed: int) -> np.ndarray:
    """``Omega`` (``nrows x ncols``) of one sweep step, as described above."""
    row = np.repeat(np.arange(nrows, dtype=np.uint64), ncols)
    col = np.tile(np.arange(ncols, dtype=np.uint64), nrows)
    zero = np.zeros_like(row)
    x = philox4x32_10([row, col, zero + np.uint64(step), zero],
                      [seed & _MASK, (seed >> 32) & _MASK])
    u1 = (x[0].astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (x[1].astype(np.float64) + 0.5) * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(nrows, ncols)


def round_bf16(x) -> np.ndarray:
    """Each value rounded to single precision, then to bfloat16 (8 significant
    bits, round to nearest, ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    u = np.where(finite, u + 0x7FFF + ((u >> 16) & 1), u) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_operands(operands: str):
    """The rounding applied to the operands of the sketch products."""
    if operands == "f64":
        return lambda v: np.asarray(v, dtype=np.float64)
    if operands == "f32":
        return lambda v: np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    if operands == "bf16":
        return round_bf16
    raise ValueError(operands)


def sketch_product(A, ell: int, step: int, seed: int, block: int = 1 << 15,
                   operands: str = "f64") -> np.ndarray:
    """``Y = A Omega`` for the ``n x ell`` test matrix of ``step``, summed over
    blocks of ``block`` rows of ``Omega`` (the same entries as
    :func:`gaussian_matrix`; only one block is drawn at a time).

    ``operands="bf16"`` (``"f32"``) rounds the entries of ``A`` and ``Omega``
    to bfloat16 (:func:`round_bf16`) or to single precision before the
    product, which is then exact in float64: the values a sketch with such
    operands multiplies."""
    rnd = round_operands(operands)
    A = rnd(np.asarray(A, dtype=np.float64))
    m, n = A.shape
    Y = np.zeros((m, ell))
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        row = np.repeat(np.arange(r0, r1, dtype=np.uint64), ell)
        col = np.tile(np.arange(ell, dtype=np.uint64), r1 - r0)
        zero = np.zeros_like(row)
        x = philox4x32_10([row, col, zero + np.uint64(step), zero],
                          [seed & _MASK, (seed >> 32) & _MASK])
        u1 = (x[0].astype(np.float64) + 0.5) * 2.0 ** -32
        u2 = (x[1].astype(np.float64) + 0.5) * 2.0 ** -32
        om = (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).reshape(r1 - r0, ell)
        Y += A[:, r0:r1] @ rnd(om)
    return Y


def range_finder(A, omega) -> np.ndarray:
    """Algorithm 4: ``Y = A Omega``, ``Q R = Y``; returns ``Q``."""
    Y = np.asarray(A, dtype=np.float64) @ omega
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def rsvd(A, Q):
    """Algorithm 5: ``B = Q^T A``, ``U~ S V^T = B``, ``U = Q U~``."""
    B = Q.T @ np.asarray(A, dtype=np.float64)
    Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
    return Q @ Ut, s, Vt


def tt_svd_sketch(a, eps: float, max_rank: int = 0, ell: int = 32, seed: int = 0,
                  return_info: bool = False, operands: str = "f64"):
    """Algorithm 1 with every truncated SVD taken by Algorithms 4 and 5.

    Same conventions as :func:`oracle.tt.tt_svd`; step ``k`` (1-based) draws
    ``Omega`` of ``n_k x ell`` entries with ``step = k`` when ``ell`` is below
    the unfolding's row count ``m_k`` and takes the exact SVD otherwise (see
    the module docstring).  ``info`` also holds ``sketched`` (the steps that
    drew ``Omega``) and ``margin``: the smallest ``|tail^2 - tau^2| / tau^2``
    over the decisions the threshold made (as in :func:`oracle.tt.tt_svd`),
    which flags rank decisions that a perturbation of ``B`` can flip.
    ``operands`` sets the values the two products of a sketched step see:
    with ``"f64"`` both are exact in float64 and the remainder is
    ``Sigma V^T`` from the SVD of ``B``; with ``"f32"`` or ``"bf16"`` the
    entries of ``A`` and ``Omega`` are rounded to that format before the
    range-finder product ``Y = A Omega``, and those of ``Q`` and ``A`` to
    single precision before ``B = Q^T A`` (each product then exact in
    float64); ``Q``, the SVD of ``B`` and ``U = Q U~`` stay in float64, and the
    remainder is the projection ``U^T A`` of the unrounded unfolding (equal to
    ``Sigma V^T`` in exact arithmetic).
    """
    v = np.asarray(a, dtype=np.float64).ravel()
    K = tt.log2_exact(v.size)
    norm = float(np.linalg.norm(v))
    info = {"norm": norm, "ranks": [1], "sv": [], "sketched": [], "margin": math.inf}
    if K == 1:
        cores = [v.reshape(1, 2, 1).copy()]
        info["ranks"].append(1)
        return (cores, info) if return_info else cores
    tau = eps * norm / math.sqrt(K - 1)
    cores = []
    r_prev = 1
    rem = v.reshape((1, -1), order="F")
    for k in range(1, K):
        A = rem.reshape((2 * r_prev, -1), order="F")
        project = False
        if ell >= A.shape[0]:
            U, s, Vt = np.linalg.svd(A, full_matrices=False)
        else:
            Q, _ = np.linalg.qr(sketch_product(A, ell, k, seed, operands=operands),
                                mode="reduced")
            if operands == "f64":
                U, s, Vt = rsvd(A, Q)
            else:
                rnd = round_operands("f32")
                Ut, s, Vt = np.linalg.svd(rnd(Q).T @ rnd(A), full_matrices=False)
                U = Q @ Ut
                project = True
            info["sketched"].append(k)
        r = tt.truncation_rank(s, tau, max_rank)
        info["sv"].append(s.copy())
        if tau > 0:
            tails = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
            r_eps = tt.truncation_rank(s, tau, 0)
            if max_rank <= 0 or r_eps <= max_rank:
                for t in [tails[r_eps]] + ([tails[r_eps - 1]] if r_eps >= 1 else []):
                    info["margin"] = min(info["margin"], abs(t - tau * tau) / (tau * tau))
        U, Vt = tt._gauge(U[:, :r].copy(), Vt[:r, :].copy())
        cores.append(U.reshape((r_prev, 2, r), order="F"))
        rem = (U.T @ A) if project else s[:r, None] * Vt
        info["ranks"].append(r)
        r_prev = r
    cores.append(rem.reshape((r_prev, 2, 1), order="F"))
    info["ranks"].append(1)
    return (cores, info) if return_info else cores
