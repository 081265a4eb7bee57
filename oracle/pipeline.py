"""The composed pipeline: decompose, convolve, round, reconstruct (Algorithm 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 2 decomposes the data and the kernel with a (modified) TT-SVD,
convolves in QTT format and retrieves the full array with Algorithm 3.  Its
Step 3 uses QTT-FFT; the path checked here replaces that step by an exact
convolution with the QTT-approximated kernel followed by TT-rounding at the
data tolerance.  Written as plain definitions:

    F  = TT-SVD_{eps, R}(x)                          (Algorithm 1 + modification (1))
    W  = TT-SVD_{eps_w}(w)        w = Toeplitz generator of the sinc kernel
    y  = T(full(W)) full(F)       exact (2.2) with the approximated kernel
    Z  = TT-SVD_{eps, R_round}(y) TT-rounding of an exact TT of y equals this
    out = full(Z)                 (Algorithm 3)

Readings: the kernel tolerance is ``eps_w = eps / 10`` unless given, the
kernel decomposition is uncapped, and rounding is uncapped unless a cap is
given.  With the singular-value drop-off of modification (3) (``delta > 0``)
the cut applies to the data decomposition and to the rounding, the
rounding standing in for the truncations inside QTT-FFT/QTT-iFFT that
Section 5 gives the same threshold; the kernel decomposition keeps its
tolerance rule.  For 2-D the image is row-major, the kernel separable, and each axis
has its own generator (column axis first in the QTT index order).
"""

from __future__ import annotations

import numpy as np

from . import conv, rsvd, tt


def relative_error(a, ref) -> float:
    """(7.1): ``||a - ref|| / ||ref||`` with the RMS norm (the ratio is the L2 ratio)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def _toeplitz(f, w, fft):
    if fft == "blocked":
        return conv.toeplitz_apply_blocked(f, w)
    return conv.toeplitz_apply_fft(f, w) if fft else conv.toeplitz_apply(f, w)


def pipeline_1d(x, B: float, eps: float, max_rank: int = 0, eps_w: float | None = None,
                round_max_rank: int = 0, fft: bool | None = None, sketch_ell: int = 0,
                sketch_seed: int = 0, delta: float = 0.0, sketch_operands: str = "f64"):
    """Run the composed pipeline on a 1-D signal of length ``2**d``.

    ``fft`` selects the DFT route for the exact convolution (default: on for
    ``d > 14``); ``fft="blocked"`` takes the direct sum as block-Toeplitz
    matrix products; all routes compute the same sum.  ``sketch_ell > 0`` takes
    the rounding's truncated SVDs from Algorithms 4 and 5 (``ell`` columns,
    ``sketch_seed``, sketch operands ``sketch_operands``: ``"f64"`` or
    ``"bf16"``); ``delta > 0`` adds the drop-off cut (exact rounding only).  Returns a dict with the cores, the intermediate full arrays,
    ranks and the output.
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    d = tt.log2_exact(x.size)
    if eps_w is None:
        eps_w = eps / 10.0
    if fft is None:
        fft = d > 14
    F, finfo = tt.tt_svd(x, eps, max_rank, return_info=True, delta=delta)
    f_t = tt.tt_full(F)
    w = conv.toeplitz_generator(d, B)
    W, winfo = tt.tt_svd(w, eps_w, 0, return_info=True)
    w_t = tt.tt_full(W)
    y = _toeplitz(f_t, w_t, fft)
    if sketch_ell > 0:
        Z, zinfo = rsvd.tt_svd_sketch(y, eps, round_max_rank, sketch_ell, sketch_seed,
                                      return_info=True, operands=sketch_operands)
    else:
        Z, zinfo = tt.tt_svd(y, eps, round_max_rank, return_info=True, delta=delta)
    out = tt.tt_full(Z)
    return dict(F=F, W=W, Z=Z, f_tilde=f_t, w=w, w_tilde=w_t, y=y, out=out,
                F_ranks=finfo["ranks"], W_ranks=winfo["ranks"], Z_ranks=zinfo["ranks"],
                F_info=finfo, W_info=winfo, Z_info=zinfo)


def pipeline_2d(img, Bx: float, By: float, eps: float, max_rank: int = 0,
                eps_w: float | None = None, round_max_rank: int = 0, fft: bool = True,
                sketch_ell: int = 0, sketch_seed: int = 0, delta: float = 0.0,
                sketch_operands: str = "f64"):
    """Run the composed pipeline on a row-major ``2**dy x 2**dx`` image
    (``sketch_*`` and ``delta`` as in :func:`pipeline_1d`)."""
    img = np.asarray(img, dtype=np.float64)
    ny, nx = img.shape
    dy, dx = tt.log2_exact(ny), tt.log2_exact(nx)
    if eps_w is None:
        eps_w = eps / 10.0
    F, finfo = tt.tt_svd(img.ravel(), eps, max_rank, return_info=True, delta=delta)
    f_t = tt.tt_full(F).reshape(ny, nx)
    wx = conv.toeplitz_generator(dx, Bx)
    wy = conv.toeplitz_generator(dy, By)
    Wx, wxinfo = tt.tt_svd(wx, eps_w, 0, return_info=True)
    Wy, wyinfo = tt.tt_svd(wy, eps_w, 0, return_info=True)
    wx_t, wy_t = tt.tt_full(Wx), tt.tt_full(Wy)
    y = conv.toeplitz_apply_2d(f_t, wy_t, wx_t, fft=fft)
    if sketch_ell > 0:
        Z, zinfo = rsvd.tt_svd_sketch(y.ravel(), eps, round_max_rank, sketch_ell, sketch_seed,
                                      return_info=True, operands=sketch_operands)
    else:
        Z, zinfo = tt.tt_svd(y.ravel(), eps, round_max_rank, return_info=True, delta=delta)
    out = tt.tt_full(Z).reshape(ny, nx)
    return dict(F=F, Wx=Wx, Wy=Wy, Z=Z, f_tilde=f_t, wx_tilde=wx_t, wy_tilde=wy_t, y=y,
                out=out, F_ranks=finfo["ranks"], Wx_ranks=wxinfo["ranks"],
                Wy_ranks=wyinfo["ranks"], Z_ranks=zinfo["ranks"], F_info=finfo, Z_info=zinfo)


def clean_reference_1d(clean, B: float) -> np.ndarray:
    """Noise-free discrete convolution (2.2) of the clean signal (reference of (7.1))."""
    clean = np.asarray(clean, dtype=np.float64).ravel()
    d = tt.log2_exact(clean.size)
    w = conv.toeplitz_generator(d, B)
    return conv.toeplitz_apply_fft(clean, w) if d > 14 else conv.toeplitz_apply(clean, w)
