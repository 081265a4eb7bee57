"""QTT-FFT convolution route (Algorithm 2, Step 3) in plain complex128 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states the route -- QFFT of the zero-padded data and kernel
tensors, their Hadamard product, QiFFT, each transform truncated by the rank
rules (1)-(3) of Section 5 with R^_max or delta^ -- but takes the QTT-FFT
itself from DKS12 without describing it.  The transform here is derived from
the radix-2 factorisation of the DFT.  With ``a = sum_p a_p 2^(p-1)`` and
``b = sum_q b_q 2^(q-1)`` (binary digits, least significant first, the QTT
index map of Section 4) and ``D`` digits,

    exp(sigma 2 pi i a b / 2^D) = prod_{q=1..D} exp(sigma 2 pi i b_q (a mod 2^m_q) / 2^m_q),
    m_q = D + 1 - q,

because ``2^(q-1) a / 2^D = a / 2^m_q`` and the digits of ``a`` above ``m_q``
only add whole turns.  Factor ``q`` involves ``b_q`` and the lowest ``m_q``
digits of ``a``, so the sum over ``a`` can be taken digit by digit from the
top (decimation in frequency): stage ``s = 1..D``, with ``m = D + 1 - s``,
sums over ``a_m`` and puts ``b_s`` at mode position ``m``:

    Y(.., b_s at m, ..) = sum_{a_m} (-1)^(a_m b_s) prod_{p<m} exp(sigma i pi b_s a_p 2^(p-m)) X(.., a_m at m, ..).

After ``D`` stages position ``p`` holds ``b_{D+1-p}``: the spectrum comes out
in bit-reversed mode order.

In TT format a stage is exact: the value of ``b_s`` travels along bonds
``1..m-1`` (which double) into cores ``1..m-1``, where it selects the
twiddle ``exp(sigma i pi 2^(p-m))`` on slice ``a_p = 1``; core ``m`` applies
the butterfly.  Bond index ``(beta, k)`` of a doubled bond is stored as
``k * r + beta``.

Readings (the paper is silent on all of these):

* Rounding inside the transform: after stage ``s`` only the bonds the stage
  doubled (``1..m-1``) are truncated.  Cores ``1..m-1`` are made
  left-orthonormal by QR, left to right, with each ``R`` absorbed into the
  next core; then a right-to-left sweep of SVDs of cores ``m..2`` (each
  viewed as ``r_{p-1} x 2 r_p``) truncates bond ``p-1`` with the rule of
  Algorithm 1 and modifications (1)/(3): ``min(r_eps, r_drop, R^_max)``, with
  ``tau = eps^ ||Y_s||_F / sqrt(D-1)``.  Cores right of ``m`` are
  right-orthonormal from the previous stage's sweep and are not touched.
  The last stage (``m = 1``) doubles nothing and is not rounded.
* QiFFT takes the spectrum in the bit-reversed order QFFT returns: the mode
  order is reversed, the same stages run with ``sigma = +1``, the order is
  reversed back and the result is scaled by ``2^-D``.
* Zero padding (Section 5 pads each dimension with at least N-1 zeros): the
  data tensor gets one more mode whose slice 1 is zero (2^(d+1) samples, the
  data in the lower half).  The kernel is the Toeplitz generator ``w`` of
  length ``2^(d+1)`` (lag ``u - 2^d`` at index ``u``) rotated by ``2^d``
  (the two slices of its top core swapped), which puts lag 0 at index 0 and
  the negative lags at the top; the lower half of the circular convolution
  is then exactly ``T(w) f``, the discrete convolution (2.2) with the shift
  used everywhere else.  The output is the slice with top digit 0.
* The Hadamard product of the two spectra has ranks ``r_F r_G``.  It is
  rounded before the inverse transform, by the randomised TT rounding
  "randomize then orthogonalize" (Al Daas, Ballard, Cazeau, Hallman,
  Miedlar, Pasha, Reid, Saibaba, SIAM J. Sci. Comput. 2023) with a Gaussian
  TT of ranks ``ell = R^_max + p``, followed by the deterministic
  right-to-left truncation with the same rule -- the randomised range finder
  of modification (2) applied to the product without forming it.  With
  ``R^_max = 0`` (no cap) the product is formed and rounded exactly instead.
* The convolution of real data is the real part of the inverse transform.
"""

from __future__ import annotations

import math

import numpy as np

from . import rsvd, tt


# ------------------------------------------------------------ basic tools
def as_complex(cores):
    return [np.asarray(c, dtype=np.complex128).copy() for c in cores]


def full(cores) -> np.ndarray:
    """Algorithm 3 (Full) for complex cores: the vector in QTT index order."""
    A = np.asarray(cores[0], dtype=np.complex128)
    A = A.reshape((-1, A.shape[2]), order="F")
    for G in cores[1:]:
        r0, _, r1 = G.shape
        A = A.reshape((-1, r0), order="F")
        A = A @ np.asarray(G, dtype=np.complex128).reshape((r0, 2 * r1), order="F")
        A = A.reshape((-1, r1), order="F")
    return A.reshape(-1, order="F")


def ranks(cores):
    return [cores[0].shape[0]] + [G.shape[2] for G in cores]


def reverse(cores):
    """The tensor with the mode order reversed: ``Z(i_1..i_D) = Y(i_D..i_1)``."""
    return [np.ascontiguousarray(np.transpose(G, (2, 1, 0))) for G in reversed(cores)]


def bit_reverse(n_bits: int) -> np.ndarray:
    """Index permutation: position ``j`` of a bit-reversed vector holds entry ``rev(j)``."""
    j = np.arange(1 << n_bits)
    r = np.zeros_like(j)
    for b in range(n_bits):
        r |= ((j >> b) & 1) << (n_bits - 1 - b)
    return r


def norm(cores) -> float:
    return float(np.linalg.norm(full(cores)))


# -------------------------------------------------------------- the stage
def fft_stage(cores, s: int, sign: int, lo: int = 0, hi: int | None = None):
    """Stage ``s`` (1-based) of the decimation-in-frequency transform of the
    digits held by cores ``lo..hi-1`` (0-based; the whole tensor by default),
    exact.  The summed digit sits at core ``m`` (1-based, ``m = lo + Dax + 1 -
    s``); cores ``lo+1..m-1`` (1-based) take the doubled bonds, the first of
    them keeps its left bond."""
    D = len(cores)
    hi = D if hi is None else hi
    m = lo + (hi - lo) + 1 - s
    out = [c.copy() for c in cores[:lo]]
    for p in range(lo + 1, m):
        G = cores[p - 1]
        r0, _, r1 = G.shape
        G1 = G.copy()
        G1[:, 1, :] *= np.exp(sign * 1j * math.pi * 2.0 ** (p - m))
        if p == lo + 1:
            H = np.concatenate([G, G1], axis=2)
        else:
            H = np.zeros((2 * r0, 2, 2 * r1), dtype=np.complex128)
            H[:r0, :, :r1] = G
            H[r0:, :, r1:] = G1
        out.append(H)
    G = cores[m - 1]
    r0, _, r1 = G.shape
    even = G[:, 0, :] + G[:, 1, :]
    odd = G[:, 0, :] - G[:, 1, :]
    if m == lo + 1:
        H = np.stack([even, odd], axis=1)
    else:
        H = np.zeros((2 * r0, 2, r1), dtype=np.complex128)
        H[:r0, 0, :] = even
        H[r0:, 1, :] = odd
    out.append(H)
    out.extend(c.copy() for c in cores[m:])
    return out


def _rank(s, tau, max_rank, delta, info):
    r = tt.truncation_rank(s, tau, max_rank)
    rd = tt.dropoff_rank(s, delta)
    if rd is not None:
        r = min(r, rd)
    if tau > 0:
        tails = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
        re = tt.truncation_rank(s, tau, 0)
        if max_rank <= 0 or re <= max_rank:
            for t in (tails[re], tails[re - 1]):
                info["margin"] = min(info["margin"], abs(t - tau * tau) / (tau * tau))
    if delta > 0:
        last = rd if rd is not None else s.size - 1
        for j in range(1, last + 1):
            if s[j - 1] > 0:
                info["delta_margin"] = min(info["delta_margin"],
                                           abs(s[j] / s[j - 1] - delta) / delta)
    if r < s.size:
        # (sigma_1, sigma_r, sigma_{r+1}) of every cut: how far the kept
        # subspace can move under a perturbation of the unfolding
        info["cuts"].append((float(s[0]), float(s[r - 1]), float(s[r])))
    return r


def _new_info():
    return {"margin": math.inf, "delta_margin": math.inf, "cuts": [], "discarded": [],
            "ranks": []}


def round_doubled(cores, m: int, eps: float, max_rank: int, delta: float, info, lo: int = 0):
    """Rounding of the bonds a stage doubled (the reading above): QR sweep over
    cores ``1..m-1`` (1-based, from the first core of the tensor), then
    truncated SVDs of cores ``m`` down to ``lo+2``, which truncate bonds
    ``m-1`` down to ``lo+1``.

    Cores right of ``m`` must be right-orthonormal.  Returns the rounded
    cores and the Frobenius norm of the discarded part (the square root of
    the discarded sigma^2, which is the rounding error exactly)."""
    G = list(cores)
    D = len(G)
    for p in range(m - 1):
        r0, _, r1 = G[p].shape
        Q, R = np.linalg.qr(G[p].reshape(r0 * 2, r1))
        k = Q.shape[1]
        G[p] = Q.reshape(r0, 2, k)
        G[p + 1] = np.einsum("kb,bjc->kjc", R, G[p + 1])
    nrm = float(np.linalg.norm(G[m - 1]))
    tau = eps * nrm / math.sqrt(D - 1) if D > 1 else 0.0
    disc = 0.0
    for p in range(m - 1, lo, -1):
        r0, _, r1 = G[p].shape
        U, s, Vh = np.linalg.svd(G[p].reshape(r0, 2 * r1), full_matrices=False)
        r = _rank(s, tau, max_rank, delta, info)
        disc += float(np.sum(s[r:] ** 2))
        G[p] = Vh[:r].reshape(r, 2, r1)
        G[p - 1] = np.einsum("aib,bc->aic", G[p - 1], U[:, :r] * s[:r])
    return G, math.sqrt(disc)


def right_orthonormalise(cores, p: int):
    """Core ``p`` (0-based) made right-orthonormal by an LQ factorisation, the
    L factor absorbed into core ``p-1``."""
    G = list(cores)
    r0, _, r1 = G[p].shape
    Q, R = np.linalg.qr(G[p].reshape(r0, 2 * r1).conj().T)   # C^H = Q R, C = R^H Q^H
    G[p] = Q.conj().T.reshape(Q.shape[1], 2, r1)
    G[p - 1] = np.einsum("aib,bc->aic", G[p - 1], R.conj().T)
    return G


def qfft(cores, sign: int = -1, eps: float = 0.0, max_rank: int = 0, delta: float = 0.0,
         return_info: bool = False, blocks=None):
    """QTT-FFT: the DFT ``X(b) = sum_a x(a) exp(sign 2 pi i a b / 2^D)`` of the
    tensor, each stage followed by the rounding of the doubled bonds; the
    result is in bit-reversed mode order.  ``eps = 0``, ``max_rank = 0`` and
    ``delta = 0`` give the exact transform (ranks up to the full ones).

    ``blocks`` (list of 0-based ``(lo, hi)`` core ranges, one per axis, in
    mode order) gives the multi-dimensional DFT: each block is transformed
    on its own digits, bit-reversed inside the block.  Blocks run right to
    left; before a block, the first core of the block to its right is made
    right-orthonormal (it carried the last butterfly), so that the rounding
    of every stage sees right-orthonormal cores right of its centre."""
    G = as_complex(cores)
    D = len(G)
    blocks = [(0, D)] if blocks is None else list(blocks)
    info = _new_info()
    for bi in range(len(blocks) - 1, -1, -1):
        lo, hi = blocks[bi]
        if bi < len(blocks) - 1:
            G = right_orthonormalise(G, blocks[bi + 1][0])
        for s in range(1, hi - lo + 1):
            m = lo + (hi - lo) + 1 - s
            G = fft_stage(G, s, sign, lo, hi)
            if m > lo + 1:
                G, e = round_doubled(G, m, eps, max_rank, delta, info, lo)
            else:
                e = 0.0
            info["discarded"].append(e)
            info["ranks"].append(ranks(G))
    return (G, info) if return_info else G


def qifft(cores, eps: float = 0.0, max_rank: int = 0, delta: float = 0.0,
          return_info: bool = False, blocks=None):
    """QTT-iFFT of a spectrum in bit-reversed mode order (per block); natural
    order result ``x(a) = 2^-D sum_b X(b) exp(+2 pi i a b / 2^D)``.  Reversing
    the whole tensor restores the natural digit order inside every block and
    mirrors the blocks, so the forward stages with the +1 exponent run on the
    mirrored blocks and the result is reversed back."""
    D = len(cores)
    mb = None if blocks is None else [(D - hi, D - lo) for lo, hi in reversed(blocks)]
    G, info = qfft(reverse(as_complex(cores)), +1, eps, max_rank, delta, True, mb)
    G = reverse(G)
    G[0] = G[0] * 2.0 ** -len(G)
    return (G, info) if return_info else G


# ------------------------------------------------------- Hadamard product
def hadamard(a, b):
    """Exact TT of the entrywise product: slice-wise Kronecker products,
    bond index ``alpha_a * r_b + alpha_b``."""
    out = []
    for A, B in zip(a, b):
        H = np.stack([np.kron(A[:, i, :], B[:, i, :]) for i in range(2)], axis=1)
        out.append(H)
    return out


def gaussian_tt(D: int, ell: int, seed: int):
    """The Gaussian sketch TT: core ``p`` (1-based) has shape
    ``(ell_{p-1}, 2, ell_p)``, ``ell_0 = ell_D = 1``, and entry ``(t, i, u)`` is
    the Philox Gaussian of the range finder with row ``2 t + i``, column ``u``
    and step ``p`` (:func:`oracle.rsvd.gaussian_matrix`)."""
    out = []
    for p in range(1, D + 1):
        l0 = 1 if p == 1 else ell
        l1 = 1 if p == D else ell
        out.append(rsvd.gaussian_matrix(2 * l0, l1, p, seed).reshape(l0, 2, l1))
    return out


def truncate_right_to_left(cores, eps: float, max_rank: int, delta: float, info):
    """Truncation sweep of a TT whose cores ``1..D-1`` are left-orthonormal:
    SVD of core ``p`` viewed as ``r_{p-1} x 2 r_p`` for ``p = D..2``."""
    G = list(cores)
    D = len(G)
    nrm = float(np.linalg.norm(G[-1]))
    tau = eps * nrm / math.sqrt(D - 1) if D > 1 else 0.0
    disc = 0.0
    for p in range(D - 1, 0, -1):
        r0, _, r1 = G[p].shape
        U, s, Vh = np.linalg.svd(G[p].reshape(r0, 2 * r1), full_matrices=False)
        r = _rank(s, tau, max_rank, delta, info)
        disc += float(np.sum(s[r:] ** 2))
        G[p] = Vh[:r].reshape(r, 2, r1)
        G[p - 1] = np.einsum("aib,bc->aic", G[p - 1], U[:, :r] * s[:r])
    return G, math.sqrt(disc)


def hadamard_round(a, b, eps: float, max_rank: int, delta: float, oversample: int = 8,
                   seed: int = 0, return_info: bool = False):
    """Rounded Hadamard product (reading above).

    With ``max_rank > 0``: sketches ``W_p`` of the right parts of the product
    with the Gaussian TT (right to left, ``W_D = 1``,
    ``W_{p-1} = sum_i H_p[:, i, :] W_p Omega_p[:, i, :]^T``), then left to
    right ``M = Z H_p`` (``Z`` the carried ``k x r`` matrix), ``Y = M W_p``,
    ``Y = Q R``, core ``p = Q``, ``Z = Q^H M``; the last core is ``Z H_D``;
    then :func:`truncate_right_to_left`.  With ``max_rank = 0``: the exact
    product, orthogonalised left to right by QR and truncated the same way."""
    H = hadamard(as_complex(a), as_complex(b))
    D = len(H)
    info = _new_info()
    if max_rank > 0:
        ell = max_rank + oversample
        Om = gaussian_tt(D, ell, seed)
        W = [None] * (D + 1)
        W[D] = np.ones((1, 1))
        for p in range(D - 1, 0, -1):
            W[p] = np.einsum("xiy,yu,tiu->xt", H[p], W[p + 1], Om[p])
        Z = np.ones((1, 1), dtype=np.complex128)
        out = []
        for p in range(D - 1):
            M = np.einsum("kx,xiy->kiy", Z, H[p])
            k = M.shape[0]
            M = M.reshape(2 * k, -1)
            Q, _ = np.linalg.qr(M @ W[p + 1])
            out.append(Q.reshape(k, 2, Q.shape[1]))
            Z = Q.conj().T @ M
        out.append(np.einsum("kx,xiy->kiy", Z, H[D - 1]))
    else:
        out = list(H)
        for p in range(D - 1):
            r0, _, r1 = out[p].shape
            Q, R = np.linalg.qr(out[p].reshape(2 * r0, r1))
            out[p] = Q.reshape(r0, 2, Q.shape[1])
            out[p + 1] = np.einsum("kb,bjc->kjc", R, out[p + 1])
    G, e = truncate_right_to_left(out, eps, max_rank, delta, info)
    info["discarded"].append(e)
    info["ranks"].append(ranks(G))
    return (G, info) if return_info else G


# ------------------------------------------------------- convolution route
def pad_data(f_cores):
    """The data tensor with one more mode whose slice 1 is zero."""
    return as_complex(f_cores) + [np.array([1.0, 0.0], dtype=np.complex128).reshape(1, 2, 1)]


def rotate_generator(w_cores):
    """The Toeplitz generator rotated by half its length (top slices swapped)."""
    G = as_complex(w_cores)
    G[-1] = np.ascontiguousarray(G[-1][:, ::-1, :])
    return G


def lower_half(cores):
    """The slice with top digit 0 (``D-1`` modes)."""
    G = list(cores[:-1])
    last = cores[-1][:, 0, 0]
    G[-1] = np.einsum("aib,b->ai", G[-1], last)[:, :, None]
    return G


def conv_fft(f_cores, w_cores, eps: float = 0.0, max_rank: int = 0, delta: float = 0.0,
             oversample: int = 8, seed: int = 0, return_info: bool = False):
    """Step 3 of Algorithm 2: ``QiFFT(QFFT(F) . QFFT(G))`` on the zero-padded
    data ``f_cores`` (``d`` modes) and the rotated Toeplitz generator
    ``w_cores`` (``d + 1`` modes), truncated by the same rule everywhere; the
    complex ``d``-mode TT of the lower half (its real part is ``T(w) f``)."""
    d = len(f_cores)
    if len(w_cores) != d + 1:
        raise ValueError("the generator needs d + 1 modes")
    Fh, i1 = qfft(pad_data(f_cores), -1, eps, max_rank, delta, True)
    Gh, i2 = qfft(rotate_generator(w_cores), -1, eps, max_rank, delta, True)
    Hh, i3 = hadamard_round(Fh, Gh, eps, max_rank, delta, oversample, seed, True)
    C, i4 = qifft(Hh, eps, max_rank, delta, True)
    y = lower_half(C)
    info = {"qfft_f": i1, "qfft_g": i2, "hadamard": i3, "qifft": i4,
            "spectra": (Fh, Gh, Hh)}
    for key in ("margin", "delta_margin"):
        info[key] = min(i[key] for i in (i1, i2, i3, i4))
    info["cuts"] = [c for i in (i1, i2, i3, i4) for c in i["cuts"]]
    return (y, info) if return_info else y


def realify(cores):
    """Real TT of the real part: interior cores ``[[Re, -Im], [Im, Re]]``
    (bond index ``s * r + alpha``), the first core's first block row, the last
    core's first block column; ranks double."""
    D = len(cores)
    if D == 1:
        return [np.real(cores[0]).copy()]
    out = []
    for p, G in enumerate(cores):
        Re, Im = np.real(G), np.imag(G)
        if p == 0:
            out.append(np.concatenate([Re, -Im], axis=2))
        elif p == D - 1:
            out.append(np.concatenate([Re, Im], axis=0))
        else:
            top = np.concatenate([Re, -Im], axis=2)
            bot = np.concatenate([Im, Re], axis=2)
            out.append(np.concatenate([top, bot], axis=0))
    return out


def pad_data_2d(f_cores, dx: int):
    """A row-major image's TT (column digits first, ``dx`` of them) with one
    zero-padding mode after the column digits (identity core, slice 1 zero)
    and one after the row digits."""
    G = as_complex(f_cores)
    r = G[dx].shape[0]
    mid = np.zeros((r, 2, r), dtype=np.complex128)
    mid[:, 0, :] = np.eye(r)
    return G[:dx] + [mid] + G[dx:] + [np.array([1.0, 0.0], dtype=np.complex128).reshape(1, 2, 1)]


def conv_fft_2d(f_cores, dx: int, wx_cores, wy_cores, eps: float = 0.0, max_rank: int = 0,
                delta: float = 0.0, oversample: int = 8, seed: int = 0, return_info: bool = False):
    """Step 3 of Algorithm 2 for a row-major image with the separable kernel:
    both axes zero-padded by one mode, the kernel the concatenated TTs of the
    two rotated Toeplitz generators (``dx + 1`` column digits, then ``dy + 1``
    row digits), the two-dimensional QFFT (one block per axis), the rounded
    Hadamard product, the QiFFT, and the slice with both padding digits 0."""
    dy = len(f_cores) - dx
    if len(wx_cores) != dx + 1 or len(wy_cores) != dy + 1:
        raise ValueError("the generators need dx + 1 and dy + 1 modes")
    blocks = [(0, dx + 1), (dx + 1, dx + dy + 2)]
    F = pad_data_2d(f_cores, dx)
    Gk = rotate_generator(wx_cores) + rotate_generator(wy_cores)
    Fh, i1 = qfft(F, -1, eps, max_rank, delta, True, blocks)
    Gh, i2 = qfft(Gk, -1, eps, max_rank, delta, True, blocks)
    Hh, i3 = hadamard_round(Fh, Gh, eps, max_rank, delta, oversample, seed, True)
    C, i4 = qifft(Hh, eps, max_rank, delta, True, blocks)
    # the padding digits at positions dx and dx + dy + 1 set to 0
    y = list(C[:dx])
    y[-1] = np.einsum("aib,bc->aic", y[-1], C[dx][:, 0, :])
    y = y + lower_half(C[dx + 1:])
    info = {"qfft_f": i1, "qfft_g": i2, "hadamard": i3, "qifft": i4}
    for key in ("margin", "delta_margin"):
        info[key] = min(i[key] for i in (i1, i2, i3, i4))
    info["cuts"] = [c for i in (i1, i2, i3, i4) for c in i["cuts"]]
    return (y, info) if return_info else y
