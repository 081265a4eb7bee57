"""qtt_full_noalloc: Full (Algorithm 3) with the library's fixed device array
instead of a caller workspace.

GPU cases call the entry point through the C-ABI binding twice in a row, the
second time on a smaller tensor (the array keeps the first call's contents),
and compare each result with qtt_full (same kernels: bit for bit) and with
the FP64 oracle's Full (1e-13 relative in FP64, 1e-5 in FP32).  The host
case checks the size limit, which is decided before anything is enqueued.
"""

import ctypes
import sys

import numpy as np
import pytest

from oracle import tt

torch = pytest.importorskip("torch")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _random_cores(d, rmax, seed, dt):
    rng = np.random.default_rng(seed)
    ranks = [1] + [int(min(rmax, 2 ** k, 2 ** (d - k), rng.integers(rmax // 2, rmax + 1)))
                   for k in range(1, d)] + [1]
    cores = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) / np.sqrt(2 * ranks[k])
             for k in range(d)]
    if dt == torch.float32:
        cores = [c.astype(np.float32).astype(np.float64) for c in cores]
    return cores


def test_noalloc_rejects_oversized_request():
    from paper_2301_13339_amd._lib import (QTT_F64, QTT_MAXD, QTT_NOALLOC_SCRATCH_MIB, lib,
                                           qtt_tensor)
    L = lib()
    d = 30
    t = qtt_tensor()
    t.d, t.dtype = d, QTT_F64
    for k in range(QTT_MAXD + 1):
        t.cap[k] = 0
    for k in range(d + 1):
        t.cap[k] = 1 if k in (0, d) else min(2 ** k, 2 ** (d - k), 64)
    need = ctypes.c_size_t()
    assert L.qtt_query_full(d, t.cap, QTT_F64, ctypes.byref(need)) == 0
    assert need.value > (QTT_NOALLOC_SCRATCH_MIB << 20)
    # non-null placeholders: the call must return before using them
    t.ranks = ctypes.c_void_p(0x1000)
    t.cores = ctypes.c_void_p(0x2000)
    t.status = None
    assert L.qtt_full_noalloc(ctypes.byref(t), ctypes.c_void_p(0x3000), None) == -2  # QTT_ENOSPC
    assert L.qtt_full_noalloc(None, ctypes.c_void_p(0x3000), None) == -1  # QTT_EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_matches_full_twice(dt):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13339_amd as q
    cases = [(20, 32, 7), (9, 6, 8)]  # second call smaller than the first
    for d, rmax, seed in cases:
        print(f"case: full_noalloc d={d} rmax={rmax} {dt}", flush=True)
        sys.stdout.flush()
        cores = _random_cores(d, rmax, seed, dt)
        t = q.from_cores(cores, dt, "cuda")
        ref_gpu = q.full(t)
        out = torch.full((1 << d,), float("nan"), dtype=dt, device="cuda")
        q.full_noalloc(t, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_gpu), "noalloc result differs from qtt_full"
        ref = tt.tt_full(cores)
        assert _rel(out.cpu().numpy(), ref) <= (1e-13 if dt == torch.float64 else 1e-5)
