"""ctypes loader and declarations for libqtt.so (mirrors include/qtt.h)."""

from __future__ import annotations

import ctypes
import os

QTT_F32 = 0
QTT_F64 = 1
QTT_C128 = 2
QTT_ROUND_EXACT = 0
QTT_ROUND_SKETCH_F32 = 1
QTT_ROUND_SKETCH_BF16 = 2
QTT_STATUS_NONFINITE = 1
QTT_STATUS_RANKCAP = 2
QTT_STATUS_FFT_RANK = 4
QTT_MAXD = 48
QTT_MAX_RANK = 64
QTT_BATCH_MAXD = 18
QTT_NOALLOC_SCRATCH_MIB = 32
QTT_FFT_MAX_RANK = 16
QTT_FFT_MAX_ELL = 32

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libqtt.so")

# every symbol include/qtt.h declares
EXPORTS = [
    "qtt_core_elems", "qtt_strerror", "qtt_last_hip_error",
    "qtt_query_decompose", "qtt_decompose", "qtt_decompose_dropoff", "qtt_kernel_sinc",
    "qtt_query_decompose_modes", "qtt_decompose_modes",
    "qtt_query_conv", "qtt_conv",
    "qtt_query_round", "qtt_round", "qtt_query_round_sketch", "qtt_round_sketch",
    "qtt_query_full", "qtt_full", "qtt_full_noalloc",
    "qtt_query_toeplitz", "qtt_toeplitz_apply",
    "qtt_query_kernel_sinc_dB", "qtt_kernel_sinc_dB",
    "qtt_query_full_adjoint", "qtt_full_adjoint",
    "qtt_query_conv_full_backward", "qtt_conv_full_backward",
    "qtt_batch_create", "qtt_batch_destroy", "qtt_batch_run", "qtt_batch_info",
    "qtt_batch_status_offset",
    "qtt_query_fft", "qtt_fft", "qtt_query_conv_fft", "qtt_conv_fft",
    "qtt_probe_start", "qtt_probe_stop",
]

# kernel classes of the launch probe (include/qtt.h)
K_CLASSES = {
    "level_gram": 1, "reduce": 2, "level_eig": 3, "project": 4, "eig_step": 5, "tail": 6,
    "conv": 7, "full_chain": 8, "full_final": 9, "other": 10, "adjoint": 11,
    "batch": 12, "sketch": 13, "sketch_gemm": 14, "qfft": 15, "qfft_hadamard": 16,
}


class QttError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


class qtt_tensor(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("cap", ctypes.c_int32 * (QTT_MAXD + 1)),
        ("ranks", ctypes.c_void_p),
        ("cores", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


_LIB = None

_I32P = ctypes.POINTER(ctypes.c_int32)
_SZP = ctypes.POINTER(ctypes.c_size_t)
_TP = ctypes.POINTER(qtt_tensor)
_VP = ctypes.c_void_p


def _declare(L):
    L.qtt_core_elems.restype = ctypes.c_size_t
    L.qtt_core_elems.argtypes = [ctypes.c_int, _I32P]
    L.qtt_strerror.restype = ctypes.c_char_p
    L.qtt_strerror.argtypes = [ctypes.c_int]
    L.qtt_last_hip_error.restype = ctypes.c_char_p
    L.qtt_last_hip_error.argtypes = []
    L.qtt_query_decompose.restype = ctypes.c_int
    L.qtt_query_decompose.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, _SZP, _SZP]
    L.qtt_decompose.restype = ctypes.c_int
    L.qtt_decompose.argtypes = [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                _TP, _VP, _VP, ctypes.c_size_t, _VP]
    L.qtt_decompose_dropoff.restype = ctypes.c_int
    L.qtt_decompose_dropoff.argtypes = [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, _TP, _VP, _VP,
                                        ctypes.c_size_t, _VP]
    L.qtt_query_decompose_modes.restype = ctypes.c_int
    L.qtt_query_decompose_modes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, _I32P, _SZP, _SZP]
    L.qtt_decompose_modes.restype = ctypes.c_int
    L.qtt_decompose_modes.argtypes = [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                      _I32P, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]
    L.qtt_kernel_sinc.restype = ctypes.c_int
    L.qtt_kernel_sinc.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_conv.restype = ctypes.c_int
    L.qtt_query_conv.argtypes = [ctypes.c_int, ctypes.c_int, _I32P, _I32P,
                                 ctypes.POINTER(_I32P), ctypes.c_int, _I32P, _SZP, _SZP]
    L.qtt_conv.restype = ctypes.c_int
    L.qtt_conv.argtypes = [_TP, _TP, ctypes.c_int, _I32P, _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_round.restype = ctypes.c_int
    L.qtt_query_round.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _I32P, _SZP, _SZP]
    L.qtt_round.restype = ctypes.c_int
    L.qtt_round.argtypes = [_TP, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                            _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_round_sketch.restype = ctypes.c_int
    L.qtt_query_round_sketch.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, _I32P, _SZP, _SZP]
    L.qtt_round_sketch.restype = ctypes.c_int
    L.qtt_round_sketch.argtypes = [_TP, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint64, _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_full.restype = ctypes.c_int
    L.qtt_query_full.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _SZP]
    L.qtt_full.restype = ctypes.c_int
    L.qtt_full.argtypes = [_TP, _VP, _VP, ctypes.c_size_t, _VP]
    L.qtt_full_noalloc.restype = ctypes.c_int
    L.qtt_full_noalloc.argtypes = [_TP, _VP, _VP]
    L.qtt_query_toeplitz.restype = ctypes.c_int
    L.qtt_query_toeplitz.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _SZP]
    L.qtt_toeplitz_apply.restype = ctypes.c_int
    L.qtt_toeplitz_apply.argtypes = [_TP, _VP, _VP, ctypes.c_int, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_kernel_sinc_dB.restype = ctypes.c_int
    L.qtt_query_kernel_sinc_dB.argtypes = [ctypes.c_int, ctypes.c_int, _I32P, _SZP, _SZP]
    L.qtt_kernel_sinc_dB.restype = ctypes.c_int
    L.qtt_kernel_sinc_dB.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_full_adjoint.restype = ctypes.c_int
    L.qtt_query_full_adjoint.argtypes = [ctypes.c_int, _I32P, ctypes.c_int, _SZP]
    L.qtt_full_adjoint.restype = ctypes.c_int
    L.qtt_full_adjoint.argtypes = [_TP, _VP, _TP, _VP, ctypes.c_size_t, _VP]
    L.qtt_query_conv_full_backward.restype = ctypes.c_int
    L.qtt_query_conv_full_backward.argtypes = [ctypes.c_int, _I32P, _I32P, _I32P, ctypes.c_int,
                                               ctypes.c_int, _SZP]
    L.qtt_conv_full_backward.restype = ctypes.c_int
    L.qtt_conv_full_backward.argtypes = [_TP, _TP, _TP, _VP, _TP, _TP, _VP, _VP, ctypes.c_size_t,
                                         _VP]
    L.qtt_batch_create.restype = ctypes.c_int
    L.qtt_batch_create.argtypes = [ctypes.c_int, _I32P, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                   _SZP]
    L.qtt_batch_destroy.restype = ctypes.c_int
    L.qtt_batch_destroy.argtypes = [_VP]
    L.qtt_batch_run.restype = ctypes.c_int
    L.qtt_batch_run.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_size_t, ctypes.c_int, _VP]
    _I64P = ctypes.POINTER(ctypes.c_int64)
    L.qtt_batch_info.restype = ctypes.c_int
    L.qtt_batch_info.argtypes = [_VP, ctypes.c_int, ctypes.c_int, _I64P, _I64P, _I32P, _I64P]
    L.qtt_batch_status_offset.restype = ctypes.c_int
    L.qtt_batch_status_offset.argtypes = [_VP, _I64P, _I32P]
    L.qtt_query_fft.restype = ctypes.c_int
    L.qtt_query_fft.argtypes = [ctypes.c_int, ctypes.c_int, _I32P, _SZP]
    L.qtt_fft.restype = ctypes.c_int
    L.qtt_fft.argtypes = [_TP, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, _TP,
                          _VP, ctypes.c_size_t, _VP]
    L.qtt_query_conv_fft.restype = ctypes.c_int
    L.qtt_query_conv_fft.argtypes = [ctypes.c_int, ctypes.c_int, _I32P, ctypes.c_int, ctypes.c_int,
                                     _I32P, _SZP]
    L.qtt_conv_fft.restype = ctypes.c_int
    L.qtt_conv_fft.argtypes = [_TP, _TP, ctypes.c_int, _I32P, ctypes.c_double, ctypes.c_int,
                               ctypes.c_double, ctypes.c_int, ctypes.c_uint64, _TP, _VP,
                               ctypes.c_size_t, _VP]
    L.qtt_probe_start.restype = ctypes.c_int
    L.qtt_probe_start.argtypes = [ctypes.c_int, ctypes.c_int]
    L.qtt_probe_stop.restype = ctypes.c_int
    L.qtt_probe_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]


def lib():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise RuntimeError(
                f"{lib_path} is missing: build it with `python -m paper_2301_13339_amd.build`")
        L = ctypes.CDLL(lib_path)
        _declare(L)
        _LIB = L
    return _LIB
