"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, sizes its workspaces and rejects bad arguments before touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2301_13339_amd import _lib
    if not os.path.exists(_lib.lib_path):
        pytest.skip("libqtt.so not built (run __graft_entry__.build())")
    return _lib


def test_exports_every_declared_symbol():
    L = _lib()
    hdr = open(os.path.join(ROOT, "include", "qtt.h")).read()
    declared = set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(qtt_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(L.EXPORTS)
    so = L.lib()
    for name in declared:
        assert hasattr(so, name), name


def test_query_decompose_capacities():
    L = _lib()
    so = L.lib()
    for d, R in [(1, 0), (5, 0), (12, 0), (20, 32), (21, 0), (13, 3)]:
        cap = (ctypes.c_int32 * (d + 1))()
        ws = ctypes.c_size_t()
        ce = ctypes.c_size_t()
        assert so.qtt_query_decompose(d, R, L.QTT_F64, cap, ctypes.byref(ws), ctypes.byref(ce)) == 0
        eff = L.QTT_MAX_RANK if R == 0 else R
        want = [1] + [min(1 << k, 1 << (d - k), eff) for k in range(1, d)] + [1]
        if d == 1:
            want = [1, 1]
        assert list(cap) == want
        assert ce.value == sum(want[k] * 2 * want[k + 1] for k in range(d))
        assert ws.value > 0


def test_query_rejects_bad_arguments():
    L = _lib()
    so = L.lib()
    assert so.qtt_query_decompose(0, 0, L.QTT_F64, None, None, None) == -1
    assert so.qtt_query_decompose(40, 0, L.QTT_F64, None, None, None) == -1
    assert so.qtt_query_decompose(5, -1, L.QTT_F64, None, None, None) == -1
    assert so.qtt_query_decompose(5, 0, 7, None, None, None) == -1
    assert so.qtt_query_full(0, None, L.QTT_F64, None) == -1


def test_calls_validate_before_launching():
    L = _lib()
    so = L.lib()
    fake = ctypes.c_void_p(0x1000)
    t = L.qtt_tensor()
    # null input
    assert so.qtt_decompose(None, 4, L.QTT_F64, 1e-3, 0, ctypes.byref(t), None, fake, 1 << 20,
                            None) == -1
    # NaN / negative tolerance
    for eps in (float("nan"), -1.0, float("inf")):
        assert so.qtt_decompose(fake, 4, L.QTT_F64, eps, 0, ctypes.byref(t), None, fake, 1 << 20,
                                None) == -1
    # workspace too small
    cap = (ctypes.c_int32 * 5)()
    ws = ctypes.c_size_t()
    so.qtt_query_decompose(4, 0, L.QTT_F64, cap, ctypes.byref(ws), None)
    t.d, t.dtype = 4, L.QTT_F64
    for k in range(5):
        t.cap[k] = cap[k]
    t.ranks = fake
    t.cores = fake
    assert so.qtt_decompose(fake, 4, L.QTT_F64, 1e-3, 0, ctypes.byref(t), None, fake,
                            ws.value - 1, None) == -2
    # output capacity too small
    t.cap[2] = cap[2] - 1
    assert so.qtt_decompose(fake, 4, L.QTT_F64, 1e-3, 0, ctypes.byref(t), None, fake, ws.value,
                            None) == -2
    # dtype mismatch between the call and the tensor
    t.cap[2] = cap[2]
    assert so.qtt_decompose(fake, 4, L.QTT_F32, 1e-3, 0, ctypes.byref(t), None, fake, ws.value,
                            None) == -1
    # drop-off threshold outside [0, 1)
    for dl in (-0.1, 1.0, float("nan")):
        assert so.qtt_decompose_dropoff(fake, 4, L.QTT_F64, 0.0, dl, 0, ctypes.byref(t), None,
                                        fake, ws.value, None) == -1
    assert so.qtt_decompose_dropoff(None, 4, L.QTT_F64, 0.0, 0.1, 0, ctypes.byref(t), None,
                                    fake, ws.value, None) == -1
    # kernel generator: bad bandwidth
    assert so.qtt_kernel_sinc(4, 0.0, 1e-5, L.QTT_F64, ctypes.byref(t), fake, 1 << 20, None) == -1
    assert so.qtt_kernel_sinc(4, float("nan"), 1e-5, L.QTT_F64, ctypes.byref(t), fake, 1 << 20,
                              None) == -1


def test_modes_query_and_validation():
    L = _lib()
    so = L.lib()
    cap = (ctypes.c_int32 * 9)()
    ws = ctypes.c_size_t()
    ne = ctypes.c_size_t()
    assert so.qtt_query_decompose_modes(8, 10, 10, 1, 10, cap, ctypes.byref(ws),
                                        ctypes.byref(ne)) == 0
    assert list(cap) == [1, 10, 10, 10, 10, 10, 10, 10, 1]
    assert ne.value == 2 * 10 * 10 + 6 * 10 * 10 * 10
    assert ws.value >= 2 * 10 ** 8 * 8            # two remainder buffers of 10^8 doubles
    # the cap is lowered so that unfoldings keep <= 128 rows
    assert so.qtt_query_decompose_modes(4, 6, 0, 0, 0, cap, None, None) == 0
    assert list(cap)[:5] == [1, 6, 21, 6, 1]
    bad = [(0, 10, 10, 0, 0), (8, 1, 10, 0, 0), (8, 65, 10, 0, 0), (8, 10, 0, 1, 10),
           (8, 10, 10, 1, 60), (8, 10, 10, 2, 0), (10, 10, 10, 0, 0)]   # 10^10 > 2^31
    for K, M, R, meth, p in bad:
        assert so.qtt_query_decompose_modes(K, M, R, meth, p, cap, None, None) == -1, (K, M)
    fake = ctypes.c_void_p(0x1000)
    so.qtt_query_decompose_modes(3, 4, 0, 0, 0, cap, ctypes.byref(ws), None)
    # null input, NaN tolerance, short workspace, capacities other than the query's
    assert so.qtt_decompose_modes(None, 3, 4, 1e-3, 0, 0, 0, 0, cap, fake, fake, None, fake,
                                  ws.value, None) == -1
    assert so.qtt_decompose_modes(fake, 3, 4, float("nan"), 0, 0, 0, 0, cap, fake, fake, None, fake,
                                  ws.value, None) == -1
    assert so.qtt_decompose_modes(fake, 3, 4, 1e-3, 0, 0, 0, 0, cap, fake, fake, None, fake,
                                  ws.value - 1, None) == -2
    cap2 = (ctypes.c_int32 * 4)(*cap[:4])
    cap2[1] = cap[1] + 1
    assert so.qtt_decompose_modes(fake, 3, 4, 1e-3, 0, 0, 0, 0, cap2, fake, fake, None, fake,
                                  ws.value, None) == -1


def test_conv_and_round_validation():
    L = _lib()
    so = L.lib()
    fake = ctypes.c_void_p(0x1000)
    f = L.qtt_tensor()
    f.d, f.dtype = 4, L.QTT_F64
    for k, c in enumerate([1, 2, 4, 2, 1]):
        f.cap[k] = c
    f.ranks = fake
    f.cores = fake
    w = L.qtt_tensor()
    w.d, w.dtype = 4, L.QTT_F64   # must be d+1 = 5 modes
    for k, c in enumerate([1, 2, 4, 2, 1]):
        w.cap[k] = c
    w.ranks = fake
    w.cores = fake
    y = L.qtt_tensor()
    am = (ctypes.c_int32 * 1)(4)
    assert so.qtt_conv(ctypes.byref(f), ctypes.byref(w), 1, am, ctypes.byref(y), None, 0,
                       None) == -1
    # axis sizes that do not add up to d
    am2 = (ctypes.c_int32 * 2)(2, 1)
    assert so.qtt_query_conv(4, 2, am2, f.cap, None, L.QTT_F64, None, None, None) == -1
    # unknown rounding method
    ycap = (ctypes.c_int32 * 5)(1, 2, 4, 2, 1)
    assert so.qtt_query_round(4, ycap, 0, L.QTT_F64, 99, None, None, None) == -1


def test_strerror_texts():
    L = _lib()
    so = L.lib()
    assert so.qtt_strerror(0) == b"ok"
    assert b"capacity" in so.qtt_strerror(-2)
    assert b"non-finite" in so.qtt_strerror(L.QTT_STATUS_NONFINITE)


def test_probe_arguments():
    L = _lib()
    so = L.lib()
    assert so.qtt_probe_start(0, 10) == -1
    assert so.qtt_probe_start(3, 0) == -1


def test_adjoint_entry_points_validate():
    L = _lib()
    so = L.lib()
    fake = ctypes.c_void_p(0x1000)
    # generator capacities for d = 4 (5 modes)
    wcap = (ctypes.c_int32 * 6)(1, 2, 4, 4, 2, 1)
    ws = ctypes.c_size_t()
    assert so.qtt_query_toeplitz(4, wcap, L.QTT_F64, ctypes.byref(ws)) == 0
    assert ws.value == 2 * (2 * 4) * 16 * 8
    bad = (ctypes.c_int32 * 6)(1, 2, 99, 4, 2, 1)
    assert so.qtt_query_toeplitz(4, bad, L.QTT_F64, ctypes.byref(ws)) == -1
    w = L.qtt_tensor()
    w.d, w.dtype = 5, L.QTT_F64
    for k in range(6):
        w.cap[k] = wcap[k]
    w.ranks = fake
    w.cores = fake
    # transpose flag must be 0 or 1; workspace must be large enough
    assert so.qtt_toeplitz_apply(ctypes.byref(w), fake, fake, 2, fake, 1 << 20, None) == -1
    assert so.qtt_toeplitz_apply(ctypes.byref(w), fake, fake, 0, fake, 8, None) == -2
    # kernel derivative: bad bandwidth
    assert so.qtt_kernel_sinc_dB(4, -1.0, 1e-8, L.QTT_F64, ctypes.byref(w), fake, 1 << 20,
                                 None) == -1
    cap = (ctypes.c_int32 * 6)()
    assert so.qtt_query_kernel_sinc_dB(4, L.QTT_F64, cap, ctypes.byref(ws), None) == 0
    assert list(cap) == [1, 2, 4, 4, 2, 1]
    # backward: w_dB and grad_B come together; grad tensor must mirror f
    f = L.qtt_tensor()
    f.d, f.dtype = 4, L.QTT_F64
    for k, c in enumerate([1, 2, 4, 2, 1]):
        f.cap[k] = c
    f.ranks = fake
    f.cores = fake
    g = L.qtt_tensor()
    ctypes.pointer(g)[0] = f
    assert so.qtt_conv_full_backward(ctypes.byref(f), ctypes.byref(w), ctypes.byref(w), fake,
                                     ctypes.byref(g), None, None, fake, 1 << 30, None) == -1
    g.cap[2] = 3
    assert so.qtt_conv_full_backward(ctypes.byref(f), ctypes.byref(w), None, fake,
                                     ctypes.byref(g), None, None, fake, 1 << 30, None) == -1
    g.cap[2] = 4
    assert so.qtt_conv_full_backward(ctypes.byref(f), ctypes.byref(w), None, fake,
                                     ctypes.byref(g), None, None, fake, 16, None) == -2
    # the kernel-core gradient tensor must mirror w
    gw = L.qtt_tensor()
    ctypes.pointer(gw)[0] = w
    gw.cap[1] = w.cap[1] + 1
    assert so.qtt_conv_full_backward(ctypes.byref(f), ctypes.byref(w), None, fake,
                                     ctypes.byref(g), ctypes.byref(gw), None, fake, 1 << 30,
                                     None) == -1
    fcap = (ctypes.c_int32 * 5)(1, 2, 4, 2, 1)
    assert so.qtt_query_conv_full_backward(4, fcap, wcap, None, 0, L.QTT_F64,
                                           ctypes.byref(ws)) == 0
    assert ws.value > 0
    ws_w = ctypes.c_size_t()
    assert so.qtt_query_conv_full_backward(4, fcap, wcap, None, 1, L.QTT_F64,
                                           ctypes.byref(ws_w)) == 0
    # the stored forward states: 2 w_cap[k] 2^d doubles for k = 1..d
    assert ws_w.value - ws.value >= sum(2 * wcap[k] * 16 * 8 for k in range(1, 5))
    assert so.qtt_query_conv_full_backward(4, fcap, wcap, None, 2, L.QTT_F64,
                                           ctypes.byref(ws_w)) == -1
    assert so.qtt_query_full_adjoint(4, fcap, L.QTT_F64, ctypes.byref(ws)) == 0
