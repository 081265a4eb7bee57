"""Python binding of libqtt (include/qtt.h): QTT denoising convolution on MI355X.

Argument marshalling only: every step runs in the HIP library.  torch is
used for device memory (the caching allocator) and the current stream.  The
binding never computes on the CPU; without the built library every call
raises.

    t   = decompose(x, eps, max_rank)      # Algorithm 1 (+ modification (1))
    w   = kernel_sinc(d, B, eps_w)         # QTT of the sinc Toeplitz generator
    y   = conv(t, [w])                     # exact (2.2) in QTT format
    z   = round(y, eps)                    # TT-rounding
    out = full(z)                          # Algorithm 3

Adjoint at fixed ranks: ``conv_full(t, B)`` is ``T(w(B)) full(t)`` as a
torch.autograd.Function whose backward calls ``qtt_conv_full_backward``.
"""

from __future__ import annotations

import ctypes
import os

import torch

from ._lib import (QTT_C128, QTT_F32, QTT_F64, QTT_FFT_MAX_ELL, QTT_FFT_MAX_RANK,
                   QTT_MAX_RANK, QTT_MAXD, QTT_ROUND_EXACT,
                   QTT_ROUND_SKETCH_BF16, QTT_ROUND_SKETCH_F32, QTT_STATUS_NONFINITE,
                   QTT_STATUS_RANKCAP, QttError, lib, lib_path, qtt_tensor)

__all__ = [
    "QTT", "probe", "from_cores", "decompose", "kernel_sinc", "conv", "round", "full", "pipeline",
    "toeplitz_apply", "kernel_sinc_dB", "full_adjoint", "conv_full_backward", "ConvFull",
    "conv_full", "Batch", "lib_path", "QttError", "QTT_MAX_RANK", "qfft", "conv_fft",
    "QTT_FFT_MAX_RANK",
]

_DT = {torch.float32: QTT_F32, torch.float64: QTT_F64, torch.complex128: QTT_C128}


class probe:
    """Context manager timing every launch of one kernel class with HIP events.

    ``with probe("eig_step") as p: ...`` then ``p.ms`` (summed GPU time) and
    ``p.launches``.  The events are recorded by the library on the stream the
    kernels are launched on.
    """

    def __init__(self, cls: str, max_launches: int = 100000):
        from ._lib import K_CLASSES
        self.cls = K_CLASSES[cls]
        self.max = int(max_launches)
        self.ms = 0.0
        self.launches = 0

    def __enter__(self):
        _check(lib().qtt_probe_start(self.cls, self.max), "qtt_probe_start")
        return self

    def __exit__(self, *exc):
        ms = ctypes.c_double()
        n = ctypes.c_int()
        _check(lib().qtt_probe_stop(ctypes.byref(ms), ctypes.byref(n)), "qtt_probe_stop")
        self.ms = ms.value
        self.launches = n.value
        return False
_TORCH = {QTT_F32: torch.float32, QTT_F64: torch.float64, QTT_C128: torch.complex128}


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().qtt_strerror(rc).decode()
        extra = lib().qtt_last_hip_error().decode() if rc == -4 else ""
        raise QttError(rc, f"{what}: {msg} {extra}".strip())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_SIDE = {}


def _side_stream(device) -> torch.cuda.Stream:
    """A second stream per device (default priority) for independent stages."""
    dev = torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _SIDE:
        _SIDE[idx] = torch.cuda.Stream(device=idx)
    return _SIDE[idx]


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class QTT:
    """A QTT tensor whose cores and ranks live on the GPU.

    ``cap`` are the host-side rank capacities; ``ranks`` (device int32,
    ``d+1`` entries) and ``cores`` (device, capacity-strided) are written by
    the producing call.  ``status`` collects device-side condition bits.
    """

    def __init__(self, d: int, dtype: int, cap, device):
        self.d = int(d)
        self.dtype = int(dtype)
        self.cap = [int(c) for c in cap]
        self.device = torch.device(device)
        n = int(lib().qtt_core_elems(self.d, (ctypes.c_int32 * (self.d + 1))(*self.cap)))
        # the producer writes every entry inside the actual ranks
        self.cores = torch.empty(max(n, 1), dtype=_TORCH[self.dtype], device=self.device)
        self.ranks = torch.empty(self.d + 1, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._keep = []

    # ------------------------------------------------------------ marshal
    def _c(self) -> qtt_tensor:
        t = qtt_tensor()
        t.d = self.d
        t.dtype = self.dtype
        for k in range(QTT_MAXD + 1):
            t.cap[k] = self.cap[k] if k <= self.d else 0
        t.ranks = ctypes.c_void_p(self.ranks.data_ptr())
        t.cores = ctypes.c_void_p(self.cores.data_ptr())
        t.status = ctypes.c_void_p(self.status.data_ptr())
        return t

    # ----------------------------------------------------------- inspect
    def record_stream(self, stream) -> None:
        for t in (self.cores, self.ranks, self.status, *self._keep):
            t.record_stream(stream)

    def ranks_host(self):
        return [int(v) for v in self.ranks.cpu()]

    def status_host(self) -> int:
        return int(self.status.cpu()[0])

    def core_offsets(self):
        offs, o = [], 0
        for k in range(self.d):
            offs.append(o)
            o += self.cap[k] * 2 * self.cap[k + 1]
        return offs

    def compact(self) -> "QTT":
        """A copy whose capacities equal the actual ranks (reads the ranks once)."""
        r = self.ranks_host()
        t = QTT(self.d, self.dtype, r, self.device)
        offs = self.core_offsets()
        o = 0
        for k in range(self.d):
            n = r[k] * 2 * r[k + 1]
            t.cores[o:o + n].copy_(self.cores[offs[k]:offs[k] + n])
            o += n
        t.ranks.copy_(self.ranks)
        t.status.copy_(self.status)
        return t

    def core_list(self):
        """Cores as CPU float64 (complex128 for complex tensors) numpy arrays of
        shape ``(r_{k-1}, 2, r_k)``."""
        r = self.ranks_host()
        flat = self.cores.detach().cpu()
        flat = (flat if flat.is_complex() else flat.double()).numpy()
        out = []
        for k, o in enumerate(self.core_offsets()):
            n = r[k] * 2 * r[k + 1]
            out.append(flat[o:o + n].reshape(r[k], 2, r[k + 1]).copy())
        return out


def _make(d, dtype, cap, device) -> QTT:
    return QTT(d, dtype, cap, device)


def from_cores(cores, dtype=torch.float64, device="cuda") -> QTT:
    """Upload host cores ``(r_{k-1}, 2, r_k)`` (capacities = their ranks)."""
    d = len(cores)
    ranks = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
    t = _make(d, _DT[dtype], ranks, device)
    wide = torch.complex128 if dtype == torch.complex128 else torch.float64
    flat = torch.cat([torch.as_tensor(c, dtype=wide).reshape(-1) for c in cores])
    t.cores[: flat.numel()].copy_(flat.to(dtype))
    t.ranks.copy_(torch.tensor(ranks, dtype=torch.int32))
    return t


def decompose(x: torch.Tensor, eps: float, max_rank: int = 0, return_sv: bool = False,
              delta: float = 0.0):
    """TT-SVD of the QTT reshape of ``x`` (length ``2**d``; images row-major).

    ``delta > 0`` adds the singular-value drop-off cut of modification (3) of
    Section 5 (``qtt_decompose_dropoff``); ``eps = 0`` with it gives the
    drop-off rule alone.
    """
    if not x.is_cuda:
        raise ValueError("decompose expects a device tensor")
    x = x.contiguous().reshape(-1)
    n = x.numel()
    d = n.bit_length() - 1
    if n < 2 or (1 << d) != n:
        raise ValueError("length must be a power of two >= 2")
    dt = _DT[x.dtype]
    cap = (ctypes.c_int32 * (d + 1))()
    ws = ctypes.c_size_t()
    _check(lib().qtt_query_decompose(d, int(max_rank), dt, cap, ctypes.byref(ws), None),
           "qtt_query_decompose")
    out = _make(d, dt, list(cap), x.device)
    w = _workspace(ws.value, x.device)
    sv = None
    if return_sv:
        sv = torch.zeros((max(d - 1, 1), 2 * QTT_MAX_RANK), dtype=torch.float64, device=x.device)
    t = out._c()
    svp = ctypes.c_void_p(sv.data_ptr()) if sv is not None else None
    if delta:
        _check(lib().qtt_decompose_dropoff(ctypes.c_void_p(x.data_ptr()), d, dt, float(eps),
                                           float(delta), int(max_rank), ctypes.byref(t), svp,
                                           ctypes.c_void_p(w.data_ptr()), ws.value,
                                           _stream(x.device)),
               "qtt_decompose_dropoff")
    else:
        _check(lib().qtt_decompose(ctypes.c_void_p(x.data_ptr()), d, dt, float(eps), int(max_rank),
                                   ctypes.byref(t), svp, ctypes.c_void_p(w.data_ptr()), ws.value,
                                   _stream(x.device)),
               "qtt_decompose")
    out._keep = [w, x]
    return (out, sv) if return_sv else out


class TTModes:
    """A TT with K modes of size M (FP64): flat ``cores`` at the query's
    capacity offsets, ``ranks`` (K+1 int32) and the ``status`` word on the
    device."""

    def __init__(self, K: int, M: int, cap, device):
        self.K, self.M, self.cap = K, M, list(cap)
        self.device = torch.device(device)
        n = sum(self.cap[k] * M * self.cap[k + 1] for k in range(K))
        self.cores = torch.zeros(n, dtype=torch.float64, device=self.device)
        self.ranks = torch.zeros(K + 1, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)

    def ranks_host(self):
        return [int(v) for v in self.ranks.cpu()]

    def status_host(self) -> int:
        return int(self.status.cpu()[0])

    def core_list(self):
        """Cores as CPU float64 arrays of shape ``(r_{k-1}, M, r_k)``."""
        r = self.ranks_host()
        flat = self.cores.cpu().numpy()
        out, off = [], 0
        for k in range(self.K):
            n = r[k] * self.M * r[k + 1]
            out.append(flat[off:off + n].reshape(r[k], self.M, r[k + 1]).copy())
            off += self.cap[k] * self.M * self.cap[k + 1]
        return out


def decompose_modes(x: torch.Tensor, M: int, eps: float, max_rank: int = 0, method: str = "svd",
                    oversample: int = 10, seed: int = 0) -> TTModes:
    """TT-SVD (``method="svd"``) or max-rank TT-RSVD (``"rsvd"``) of ``x`` read as a
    tensor with modes of size ``M`` (``x.numel() == M**K``, first mode fastest)."""
    if not x.is_cuda or x.dtype != torch.float64:
        raise ValueError("decompose_modes expects a float64 device tensor")
    x = x.contiguous().reshape(-1)
    K, n = 0, 1
    while n < x.numel():
        n *= M
        K += 1
    if n != x.numel() or K < 1:
        raise ValueError("the length must be a power of the mode size")
    meth = {"svd": 0, "rsvd": 1}[method]
    cap = (ctypes.c_int32 * (K + 1))()
    ws = ctypes.c_size_t()
    _check(lib().qtt_query_decompose_modes(K, int(M), int(max_rank), meth, int(oversample), cap,
                                           ctypes.byref(ws), None), "qtt_query_decompose_modes")
    out = TTModes(K, int(M), list(cap), x.device)
    w = _workspace(ws.value, x.device)
    _check(lib().qtt_decompose_modes(ctypes.c_void_p(x.data_ptr()), K, int(M), float(eps),
                                     int(max_rank), meth, int(oversample), ctypes.c_uint64(seed),
                                     cap, ctypes.c_void_p(out.ranks.data_ptr()),
                                     ctypes.c_void_p(out.cores.data_ptr()),
                                     ctypes.c_void_p(out.status.data_ptr()),
                                     ctypes.c_void_p(w.data_ptr()), ws.value, _stream(x.device)),
           "qtt_decompose_modes")
    out._keep = [w, x]
    return out


def kernel_sinc(d: int, B: float, eps_w: float, dtype=torch.float64, device="cuda") -> QTT:
    """QTT (``d+1`` modes) of the normalised sinc Toeplitz generator of a ``2**d`` grid."""
    dt = _DT[dtype]
    cap = (ctypes.c_int32 * (d + 2))()
    ws = ctypes.c_size_t()
    _check(lib().qtt_query_decompose(d + 1, 0, dt, cap, ctypes.byref(ws), None),
           "qtt_query_decompose")
    dev = torch.device(device)
    out = _make(d + 1, dt, list(cap), dev)
    w = _workspace(ws.value, dev)
    t = out._c()
    _check(lib().qtt_kernel_sinc(int(d), float(B), float(eps_w), dt, ctypes.byref(t),
                                 ctypes.c_void_p(w.data_ptr()), ws.value, _stream(dev)),
           "qtt_kernel_sinc")
    out._keep = [w]
    return out


def conv(f: QTT, w, axis_modes=None) -> QTT:
    """Exact convolution in QTT format with one kernel per axis (column axis first)."""
    ws_list = list(w)
    n_axes = len(ws_list)
    if axis_modes is None:
        axis_modes = [f.d] if n_axes == 1 else None
    if axis_modes is None:
        raise ValueError("axis_modes required for images")
    am = (ctypes.c_int32 * n_axes)(*axis_modes)
    fcap = (ctypes.c_int32 * (f.d + 1))(*f.cap)
    wcaps = [(ctypes.c_int32 * (t.d + 1))(*t.cap) for t in ws_list]
    wcp = (ctypes.POINTER(ctypes.c_int32) * n_axes)(
        *[ctypes.cast(c, ctypes.POINTER(ctypes.c_int32)) for c in wcaps])
    ycap = (ctypes.c_int32 * (f.d + 1))()
    wsb = ctypes.c_size_t()
    _check(lib().qtt_query_conv(f.d, n_axes, am, fcap, wcp, f.dtype, ycap, ctypes.byref(wsb), None),
           "qtt_query_conv")
    y = _make(f.d, f.dtype, list(ycap), f.device)
    warr = (qtt_tensor * n_axes)(*[t._c() for t in ws_list])
    fc = f._c()
    yc = y._c()
    _check(lib().qtt_conv(ctypes.byref(fc), warr, n_axes, am, ctypes.byref(yc), None, 0,
                          _stream(f.device)), "qtt_conv")
    y._keep = [f, ws_list]
    return y


_METHODS = {"exact": QTT_ROUND_EXACT, "sketch_f32": QTT_ROUND_SKETCH_F32,
            "sketch_bf16": QTT_ROUND_SKETCH_BF16}


def round(y: QTT, eps: float, max_rank: int = 0, method: str = "exact", seed: int = 0,  # noqa: A001
          ell: int | None = None, delta: float = 0.0) -> QTT:
    """TT-rounding of ``y`` at tolerance ``eps``.

    ``method``: ``"exact"``, ``"sketch_f32"`` or ``"sketch_bf16"`` (the
    randomised form; ``ell`` columns, default ``QTT_SKETCH_ELL``).
    ``delta > 0`` (exact method only) adds the singular-value drop-off cut:
    Full of ``y`` followed by ``qtt_decompose_dropoff``, the same two stages
    ``qtt_round`` runs.
    """
    if delta:
        if method != "exact":
            raise ValueError("the drop-off cut is available for the exact rounding only")
        return decompose(full(y), eps, max_rank, delta=delta)
    m = _METHODS[method]
    ycap = (ctypes.c_int32 * (y.d + 1))(*y.cap)
    zcap = (ctypes.c_int32 * (y.d + 1))()
    wsb = ctypes.c_size_t()
    if m == QTT_ROUND_EXACT or ell is None:
        _check(lib().qtt_query_round(y.d, ycap, int(max_rank), y.dtype, m, zcap,
                                     ctypes.byref(wsb), None), "qtt_query_round")
    else:
        _check(lib().qtt_query_round_sketch(y.d, ycap, int(max_rank), y.dtype, int(ell), zcap,
                                            ctypes.byref(wsb), None), "qtt_query_round_sketch")
    z = _make(y.d, y.dtype, list(zcap), y.device)
    w = _workspace(wsb.value, y.device)
    yc, zc = y._c(), z._c()
    if m == QTT_ROUND_EXACT or ell is None:
        _check(lib().qtt_round(ctypes.byref(yc), float(eps), int(max_rank), m,
                               ctypes.c_uint64(seed), ctypes.byref(zc),
                               ctypes.c_void_p(w.data_ptr()), wsb.value, _stream(y.device)),
               "qtt_round")
    else:
        _check(lib().qtt_round_sketch(ctypes.byref(yc), float(eps), int(max_rank), int(ell),
                                      int(m == QTT_ROUND_SKETCH_BF16), ctypes.c_uint64(seed),
                                      ctypes.byref(zc), ctypes.c_void_p(w.data_ptr()), wsb.value,
                                      _stream(y.device)), "qtt_round_sketch")
    z._keep = [w, y]
    return z


def full(t: QTT, out: torch.Tensor | None = None) -> torch.Tensor:
    """Algorithm 3: the ``2**d`` entries of ``t`` (QTT index order)."""
    cap = (ctypes.c_int32 * (t.d + 1))(*t.cap)
    wsb = ctypes.c_size_t()
    _check(lib().qtt_query_full(t.d, cap, t.dtype, ctypes.byref(wsb)), "qtt_query_full")
    if out is None:
        out = torch.empty(1 << t.d, dtype=_TORCH[t.dtype], device=t.device)
    w = _workspace(wsb.value, t.device)
    tc = t._c()
    _check(lib().qtt_full(ctypes.byref(tc), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(w.data_ptr()), wsb.value, _stream(t.device)),
           "qtt_full")
    t._keep = t._keep + [w]
    return out


def full_noalloc(t: QTT, out: torch.Tensor) -> torch.Tensor:
    """``full`` through ``qtt_full_noalloc``: no workspace, the library's fixed
    device array holds the interface matrices (``out`` is the caller's)."""
    if out.numel() != (1 << t.d) or out.dtype != _TORCH[t.dtype] or not out.is_contiguous():
        raise ValueError("out must be a contiguous array of 2**d elements of the tensor's dtype")
    tc = t._c()
    _check(lib().qtt_full_noalloc(ctypes.byref(tc), ctypes.c_void_p(out.data_ptr()),
                                  _stream(t.device)), "qtt_full_noalloc")
    return out


def qfft(x: QTT, inverse: bool = False, eps: float = 0.0, max_rank: int = 0,
         delta: float = 0.0) -> QTT:
    """QTT-FFT of a complex QTT (bit-reversed output), or with ``inverse`` the
    QTT-iFFT of a bit-reversed spectrum; every stage rounded by the rule
    ``(eps, max_rank, delta)`` (see ``qtt_fft`` in include/qtt.h)."""
    if x.dtype != QTT_C128:
        raise ValueError("qfft takes a complex QTT (torch.complex128 cores)")
    cap = (ctypes.c_int32 * (x.d + 1))()
    ws = ctypes.c_size_t()
    _check(lib().qtt_query_fft(x.d, int(max_rank), cap, ctypes.byref(ws)), "qtt_query_fft")
    y = _make(x.d, QTT_C128, list(cap), x.device)
    wsb = _workspace(ws.value, x.device)
    xc, yc = x._c(), y._c()
    _check(lib().qtt_fft(ctypes.byref(xc), int(bool(inverse)), float(eps), int(max_rank),
                         float(delta), ctypes.byref(yc), ctypes.c_void_p(wsb.data_ptr()),
                         ws.value, _stream(x.device)), "qtt_fft")
    y._keep.append(wsb)
    return y


def conv_fft(f: QTT, w, max_rank_hat: int = 15, eps_hat: float = 0.0, delta_hat: float = 0.0,
             oversample: int = 8, seed: int = 0, axis_modes=None) -> QTT:
    """Step 3 of Algorithm 2 by QTT-FFT: ``QiFFT(QFFT(F) . QFFT(G))`` of the
    zero-padded data ``f`` and the rotated Toeplitz generator(s) ``w`` (one
    QTT with ``d + 1`` modes for a signal, or ``[wx, wy]`` with
    ``axis_modes = [dx, dy]`` for a row-major image, as from
    :func:`kernel_sinc`); returns the real part with the padding digits at 0
    as a real QTT (dtype of ``f``)."""
    ws_list = list(w) if isinstance(w, (list, tuple)) else [w]
    n_axes = len(ws_list)
    am = [f.d] if axis_modes is None else [int(v) for v in axis_modes]
    amc = (ctypes.c_int32 * len(am))(*am)
    cap = (ctypes.c_int32 * (f.d + 1))()
    wsz = ctypes.c_size_t()
    _check(lib().qtt_query_conv_fft(f.d, n_axes, amc, int(max_rank_hat), int(oversample), cap,
                                    ctypes.byref(wsz)), "qtt_query_conv_fft")
    y = _make(f.d, f.dtype, list(cap), f.device)
    wsb = _workspace(wsz.value, f.device)
    fc, yc = f._c(), y._c()
    warr = (qtt_tensor * n_axes)(*[t._c() for t in ws_list])
    _check(lib().qtt_conv_fft(ctypes.byref(fc), warr, n_axes, amc, float(eps_hat),
                              int(max_rank_hat), float(delta_hat), int(oversample),
                              ctypes.c_uint64(int(seed)), ctypes.byref(yc),
                              ctypes.c_void_p(wsb.data_ptr()), wsz.value, _stream(f.device)),
           "qtt_conv_fft")
    y._keep.append(wsb)
    return y


def pipeline_fft(x: torch.Tensor, B, eps: float, max_rank: int = 10,
                 max_rank_hat: int = 15, eps_w: float | None = None, eps_hat: float = 0.0,
                 delta: float = 0.0, oversample: int = 8, seed: int = 0, shape2d=None):
    """Algorithm 2 with the QTT-FFT route of Step 3: decompose (tolerance, cap
    ``max_rank``, optional drop-off), build the kernel QTT(s), convolve by
    ``QiFFT(QFFT(F) . QFFT(G))`` truncated at ``max_rank_hat`` (and ``delta``,
    as the paper uses the same threshold in both places), reconstruct.  ``B``
    is one bandwidth, or ``(Bx, By)`` with ``shape2d = (ny, nx)`` for a
    row-major image.  Returns ``(out, stages)``."""
    if eps_w is None:
        eps_w = eps / 10.0
    d = int(x.numel()).bit_length() - 1
    main = torch.cuda.current_stream(x.device)
    side = _side_stream(x.device)
    side.wait_stream(main)
    f = decompose(x, eps, max_rank, delta=delta)
    with torch.cuda.stream(side):
        if shape2d is None:
            w = [kernel_sinc(d, float(B), eps_w, x.dtype, x.device)]
            am = None
        else:
            ny, nx = shape2d
            dy, dx = ny.bit_length() - 1, nx.bit_length() - 1
            bx, by = B
            w = [kernel_sinc(dx, float(bx), eps_w, x.dtype, x.device),
                 kernel_sinc(dy, float(by), eps_w, x.dtype, x.device)]
            am = [dx, dy]
    main.wait_stream(side)
    for t in w:
        t.record_stream(main)
    y = conv_fft(f, w, max_rank_hat, eps_hat, delta, oversample, seed, am)
    out = full(y)
    if shape2d is not None:
        out = out.reshape(shape2d)
    return out, dict(f=f, w=w, y=y)


def pipeline(x: torch.Tensor, B, eps: float, max_rank: int = 0, eps_w: float | None = None,
             round_method: str = "exact", round_max_rank: int = 0, shape2d=None,
             sketch_ell: int | None = None, sketch_seed: int = 0, delta: float = 0.0):
    """Decompose, build the kernel QTT, convolve, round and reconstruct.

    ``B`` is one bandwidth (signal) or ``(Bx, By)`` with ``shape2d = (ny, nx)``
    for a row-major image.  ``delta > 0`` applies the singular-value drop-off
    cut to the data decomposition and to the rounding.  Returns ``(out,
    stages)``.
    """
    if eps_w is None:
        eps_w = eps / 10.0
    dt = x.dtype
    # the kernel QTT does not depend on the samples: build it on a side
    # stream while the signal is decomposed on the current one.  The signal's
    # sweep is the longer chain, so its launches are issued first (launching
    # the kernel QTT first would hold the signal back by the host time of
    # those launches).
    main = torch.cuda.current_stream(x.device)
    side = _side_stream(x.device)
    side.wait_stream(main)
    f = decompose(x, eps, max_rank, delta=delta)
    with torch.cuda.stream(side):
        if shape2d is None:
            w = [kernel_sinc(int(x.numel()).bit_length() - 1, float(B), eps_w, dt, x.device)]
        else:
            ny, nx = shape2d
            dy, dx = ny.bit_length() - 1, nx.bit_length() - 1
            bx, by = B
            w = [kernel_sinc(dx, float(bx), eps_w, dt, x.device),
                 kernel_sinc(dy, float(by), eps_w, dt, x.device)]
    main.wait_stream(side)
    for t in w:
        t.record_stream(main)
    am = [f.d] if shape2d is None else [dx, dy]
    y = conv(f, w, am)
    z = round(y, eps, round_max_rank, round_method, sketch_seed, sketch_ell, delta=delta)
    out = full(z)
    if shape2d is not None:
        out = out.reshape(shape2d)
    return out, dict(f=f, w=w, y=y, z=z)


class PipelineGraph:
    """``pipeline`` captured once into a HIP graph and replayed.

    Every launch of the pipeline (both streams, all stages) is recorded on
    the first call after an eager warm-up; ``run()`` replays the graph, so a
    step costs one launch on the host.  ``x`` is the captured input buffer:
    copy new samples into it (same shape and dtype) before ``run()``.  The
    outputs (``out``, ``stages``) are the captured tensors, rewritten by
    every replay.
    """

    def __init__(self, x: torch.Tensor, B, eps: float, max_rank: int = 0, **kw):
        self.x = x
        # warm-up: first-call kernel attributes, workspace sizes, side stream
        pipeline(x, B, eps, max_rank, **kw)
        torch.cuda.synchronize(x.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out, self.stages = pipeline(x, B, eps, max_rank, **kw)
        torch.cuda.synchronize(x.device)

    def run(self) -> torch.Tensor:
        self.graph.replay()
        return self.out


# ------------------------------------------------------------------ adjoint
def toeplitz_apply(w: QTT, x: torch.Tensor, transpose: bool = False,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """``T(w) x`` (or ``T(w)^T x``) for a full vector ``x`` of ``2**(w.d-1)`` entries."""
    d = w.d - 1
    if x.dtype != _TORCH[w.dtype] or x.numel() != (1 << d) or not x.is_contiguous():
        raise QttError(-1, "toeplitz_apply: x must be contiguous with 2^d entries of w's dtype")
    cap = (ctypes.c_int32 * (w.d + 1))(*w.cap)
    wsb = ctypes.c_size_t()
    _check(lib().qtt_query_toeplitz(d, cap, w.dtype, ctypes.byref(wsb)), "qtt_query_toeplitz")
    if out is None:
        out = torch.empty_like(x)
    ws = _workspace(wsb.value, x.device)
    wc = w._c()
    _check(lib().qtt_toeplitz_apply(ctypes.byref(wc), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), int(bool(transpose)),
                                    ctypes.c_void_p(ws.data_ptr()), wsb.value, _stream(x.device)),
           "qtt_toeplitz_apply")
    return out


def kernel_sinc_dB(d: int, B: float, eps_w: float, dtype=torch.float64, device="cuda") -> QTT:
    """QTT (``d+1`` modes) of the bandwidth derivative of the normalised generator."""
    dt = _DT[dtype]
    cap = (ctypes.c_int32 * (d + 2))()
    ws = ctypes.c_size_t()
    _check(lib().qtt_query_kernel_sinc_dB(int(d), dt, cap, ctypes.byref(ws), None),
           "qtt_query_kernel_sinc_dB")
    dev = torch.device(device)
    out = _make(d + 1, dt, list(cap), dev)
    w = _workspace(ws.value, dev)
    t = out._c()
    _check(lib().qtt_kernel_sinc_dB(int(d), float(B), float(eps_w), dt, ctypes.byref(t),
                                    ctypes.c_void_p(w.data_ptr()), ws.value, _stream(dev)),
           "qtt_kernel_sinc_dB")
    out._keep = [w]
    return out


def _grad_like(f: QTT) -> QTT:
    g = _make(f.d, f.dtype, f.cap, f.device)
    g.cores.zero_()
    return g


def full_adjoint(f: QTT, g: torch.Tensor) -> QTT:
    """Cores of ``d<g, full(f)>/d f_k`` (same ranks and capacities as ``f``)."""
    cap = (ctypes.c_int32 * (f.d + 1))(*f.cap)
    wsb = ctypes.c_size_t()
    _check(lib().qtt_query_full_adjoint(f.d, cap, f.dtype, ctypes.byref(wsb)),
           "qtt_query_full_adjoint")
    gr = _grad_like(f)
    ws = _workspace(wsb.value, f.device)
    fc, gc = f._c(), gr._c()
    _check(lib().qtt_full_adjoint(ctypes.byref(fc), ctypes.c_void_p(g.data_ptr()),
                                  ctypes.byref(gc), ctypes.c_void_p(ws.data_ptr()), wsb.value,
                                  _stream(f.device)), "qtt_full_adjoint")
    return gr


def conv_full_backward(f: QTT, w: QTT, w_dB: QTT | None, grad_y: torch.Tensor,
                       grad_w: bool = False):
    """``(grad_f, grad_w, grad_B)`` of ``y = T(w) full(f) = full(conv(f, w))`` for the
    upstream gradient ``grad_y``; ``grad_w`` (the kernel cores) only when asked
    for, ``grad_B`` only with ``w_dB``.  For ``grad_w`` pass a compact ``w``
    (``w.compact()``): the workspace keeps d states sized by its capacities."""
    if grad_y.dtype != _TORCH[f.dtype] or grad_y.numel() != (1 << f.d):
        raise QttError(-1, "conv_full_backward: grad_y must have 2^d entries of f's dtype")
    grad_y = grad_y.contiguous()
    fcap = (ctypes.c_int32 * (f.d + 1))(*f.cap)
    wcap = (ctypes.c_int32 * (w.d + 1))(*w.cap)
    bcap = (ctypes.c_int32 * (w_dB.d + 1))(*w_dB.cap) if w_dB is not None else None
    wsb = ctypes.c_size_t()
    _check(lib().qtt_query_conv_full_backward(f.d, fcap, wcap, bcap, int(bool(grad_w)), f.dtype,
                                              ctypes.byref(wsb)),
           "qtt_query_conv_full_backward")
    gr = _grad_like(f)
    gw = _grad_like(w) if grad_w else None
    gB = torch.zeros(1, dtype=torch.float64, device=f.device) if w_dB is not None else None
    ws = _workspace(wsb.value, f.device)
    fc, wc, gc = f._c(), w._c(), gr._c()
    gwc = gw._c() if gw is not None else None
    bc = w_dB._c() if w_dB is not None else None
    _check(lib().qtt_conv_full_backward(
        ctypes.byref(fc), ctypes.byref(wc), ctypes.byref(bc) if bc is not None else None,
        ctypes.c_void_p(grad_y.data_ptr()), ctypes.byref(gc),
        ctypes.byref(gwc) if gwc is not None else None,
        ctypes.c_void_p(gB.data_ptr()) if gB is not None else None,
        ctypes.c_void_p(ws.data_ptr()), wsb.value, _stream(f.device)), "qtt_conv_full_backward")
    return gr, gw, gB


def _with_cores(template: QTT, cores: torch.Tensor) -> QTT:
    t = QTT.__new__(QTT)
    t.d, t.dtype, t.cap, t.device = template.d, template.dtype, list(template.cap), template.device
    t.cores = cores.detach()
    t.ranks = template.ranks
    t.status = template.status
    t._keep = []
    return t


class ConvFull(torch.autograd.Function):
    """``y = full(conv(F, W)) = T(w) full(F)`` at fixed ranks, differentiable in the
    signal cores, the kernel cores and the bandwidth ``B``.

    ``forward(cores, wcores, B, template, wtemplate, eps_dB)``: ``cores`` and
    ``wcores`` are the flat capacity-strided core arrays of ``template`` (the
    signal QTT) and ``wtemplate`` (the kernel generator QTT, d+1 modes), whose
    ranks are kept; ``B`` is a one-element tensor.  The forward convolves in
    QTT format (``qtt_conv``) and reconstructs (``qtt_full``).  The backward
    recomputes ``full(F)`` instead of storing it; ``dL/dB`` takes the QTT of
    ``dw/dB`` built at ``eps_dB`` (the kernel cores are treated as the
    generator they approximate).
    """

    @staticmethod
    def forward(ctx, cores, wcores, B, template, wtemplate, eps_dB):
        f = _with_cores(template, cores)
        w = _with_cores(wtemplate, wcores)
        y = full(conv(f, [w], [f.d]))
        ctx.save_for_backward(cores, wcores, B)
        ctx.template, ctx.wtemplate, ctx.eps_dB = template, wtemplate, eps_dB
        return y

    @staticmethod
    def backward(ctx, gy):
        cores, wcores, B = ctx.saved_tensors
        f = _with_cores(ctx.template, cores)
        w = _with_cores(ctx.wtemplate, wcores)
        need_w, need_b = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        wdb = kernel_sinc_dB(f.d, float(B), ctx.eps_dB, _TORCH[f.dtype], f.device) if need_b \
            else None
        gr, gw, gB = conv_full_backward(f, w, wdb, gy.contiguous().to(_TORCH[f.dtype]),
                                        grad_w=need_w)
        gcores = gr.cores if ctx.needs_input_grad[0] else None
        gwcores = gw.cores if need_w else None
        gb = gB.to(device=B.device, dtype=B.dtype).reshape(B.shape) if need_b else None
        return gcores, gwcores, gb, None, None, None


def conv_full(f: QTT, B: torch.Tensor, cores: torch.Tensor | None = None, eps_w: float = 1e-12,
              eps_dB: float = 1e-12, w: QTT | None = None,
              wcores: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable ``full(conv(F, W))``; ``cores`` defaults to ``f.cores``; the
    kernel ``w`` defaults to ``kernel_sinc(d, B, eps_w)`` (compacted to its
    ranks) and ``wcores`` to ``w.cores``."""
    if w is None:
        w = kernel_sinc(f.d, float(B), eps_w, _TORCH[f.dtype], f.device).compact()
    return ConvFull.apply(f.cores if cores is None else cores,
                          w.cores if wcores is None else wcores, B, f, w, eps_dB)


# ------------------------------------------------------------------ batched
class Batch:
    """Many independent lines through the whole pipeline (``qtt_batch_*``).

    ``d`` and ``B`` give each line's length ``2**d[l]`` and kernel bandwidth;
    the lines are stored back to back in the input and output vectors.  The
    plan owns its workspace (a torch uint8 tensor on ``device``).
    """

    def __init__(self, d, B, dtype=torch.float32, eps: float = 1e-4, max_rank: int = 32,
                 eps_w: float | None = None, w_max_rank: int = 0, round_max_rank: int = 0,
                 device="cuda"):
        self.d = [int(v) for v in d]
        self.B = [float(v) for v in B]
        if len(self.d) != len(self.B) or not self.d:
            raise QttError(-1, "Batch: d and B must have the same non-zero length")
        self.n = len(self.d)
        self.dtype = dtype
        self.device = torch.device(device)
        self.eps_w = eps / 10.0 if eps_w is None else eps_w
        n = self.n
        dd = (ctypes.c_int32 * n)(*self.d)
        bb = (ctypes.c_double * n)(*self.B)
        plan = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        _check(lib().qtt_batch_create(n, dd, bb, _DT[dtype], float(eps), int(max_rank),
                                      float(self.eps_w), int(w_max_rank), int(round_max_rank),
                                      ctypes.byref(plan), ctypes.byref(wsb)), "qtt_batch_create")
        self._plan = plan
        self._lib = lib()
        self.ws = torch.empty(max(wsb.value, 1), dtype=torch.uint8, device=self.device)
        self.offsets = []
        o = 0
        for v in self.d:
            self.offsets.append(o)
            o += 1 << v
        self.samples = o

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            self._lib.qtt_batch_destroy(plan)
            self._plan = None

    def run(self, x: torch.Tensor, out: torch.Tensor | None = None, graph: bool = True):
        if x.dtype != self.dtype or x.numel() != self.samples or not x.is_contiguous():
            raise QttError(-1, "Batch.run: x must be contiguous with sum 2^d entries")
        if out is None:
            out = torch.empty_like(x)
        _check(self._lib.qtt_batch_run(self._plan, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                       int(bool(graph)), _stream(self.device)), "qtt_batch_run")
        return out

    def line(self, v: torch.Tensor, l: int) -> torch.Tensor:
        o = self.offsets[l]
        return v[o:o + (1 << self.d[l])]

    def _info(self, l, which):
        ro, co = ctypes.c_int64(), ctypes.c_int64()
        cap = ctypes.c_int32()
        so = ctypes.c_int64()
        _check(self._lib.qtt_batch_info(self._plan, int(l), int(which), ctypes.byref(ro),
                                        ctypes.byref(co), ctypes.byref(cap), ctypes.byref(so)),
               "qtt_batch_info")
        return ro.value, co.value, cap.value

    def ranks(self, l: int, which: int = 2):
        """Ranks of line ``l``: which = 0 signal, 1 kernel, 2 rounded."""
        ro, _, _ = self._info(l, which)
        D = self.d[l] + (1 if which == 1 else 0)
        r = self.ws[ro:ro + 4 * (D + 1)].view(torch.int32)
        return [int(v) for v in r.cpu()]

    def cores(self, l: int, which: int = 2):
        """Cores of line ``l`` as CPU float64 arrays ``(r_{k-1}, 2, r_k)``."""
        ro, co, cap = self._info(l, which)
        D = self.d[l] + (1 if which == 1 else 0)
        r = self.ranks(l, which)
        caps = [1] + [min(cap, 1 << k, 1 << (D - k)) for k in range(1, D)] + [1]
        es = 8 if self.dtype == torch.float64 else 4
        n = sum(caps[k] * 2 * caps[k + 1] for k in range(D))
        flat = self.ws[co:co + es * n].view(self.dtype).double().cpu().numpy()
        out, o = [], 0
        for k in range(D):
            m = r[k] * 2 * r[k + 1]
            out.append(flat[o:o + m].reshape(r[k], 2, r[k + 1]).copy())
            o += caps[k] * 2 * caps[k + 1]
        return out

    def status(self):
        """(3, n) status words: signal, kernel and rounding decomposition."""
        so = ctypes.c_int64()
        cb = ctypes.c_int32()
        _check(self._lib.qtt_batch_status_offset(self._plan, ctypes.byref(so), ctypes.byref(cb)),
               "qtt_batch_status_offset")
        self.chunk_bits = cb.value
        return self.ws[so.value:so.value + 12 * self.n].view(torch.int32).reshape(3, self.n).cpu()
