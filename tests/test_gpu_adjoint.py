"""GPU parity of the adjoint (Toeplitz products on full vectors, the adjoint of
Full, the bandwidth-derivative kernel QTT, the composed backward and the
autograd Function) against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import conv, grads, tt
from synthetic import generators as G

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13339_amd as qq
    return qq


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_qtt(vec, eps):
    """Cores of the oracle's TT-SVD of ``vec`` and the vector they represent."""
    cores = tt.tt_svd(vec, eps)
    return cores, tt.tt_full(cores)


TOL = {torch.float64: 1e-12, torch.float32: 2e-6}


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("d,B", [(1, 0.7), (2, 1.5), (5, 7.0), (10, 60.0), (14, 500.0)])
def test_toeplitz_apply_forward_and_transpose(q, d, B, dt):
    """The same QTT generator on both sides (oracle cores uploaded): the
    products must agree to rounding."""
    print(f"toeplitz d={d} B={B} {dt}", flush=True)
    rng = np.random.default_rng(100 + d)
    n = 1 << d
    x = rng.standard_normal(n)
    wc, wv = oracle_qtt(conv.toeplitz_generator(d, B), 1e-10)
    w = q.from_cores(wc, dt, DEV)
    xt = torch.tensor(x, dtype=dt, device=DEV)
    y = q.toeplitz_apply(w, xt).cpu().numpy()
    yt = q.toeplitz_apply(w, xt, transpose=True).cpu().numpy()
    assert rel(y, conv.toeplitz_apply(x, wv)) <= TOL[dt]
    assert rel(yt, conv.toeplitz_transpose_apply(x, wv, fft=False)) <= TOL[dt]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("d,eps,R", [(1, 0.0, 0), (3, 0.0, 0), (9, 1e-3, 8), (13, 1e-4, 16)])
def test_full_adjoint_matches_oracle(q, d, eps, R, dt):
    print(f"full_adjoint d={d} {dt}", flush=True)
    rng = np.random.default_rng(7 + d)
    cores = tt.tt_svd(rng.standard_normal(1 << d), eps, R)
    g = rng.standard_normal(1 << d)
    f = q.from_cores(cores, dt, DEV)
    gr = q.full_adjoint(f, torch.tensor(g, dtype=dt, device=DEV))
    assert gr.ranks_host() == f.ranks_host()
    ref = grads.full_adjoint(cores, g)
    got = gr.core_list()
    for k in range(d):
        assert rel(got[k], ref[k]) <= (1e-12 if dt == torch.float64 else 1e-5), k


@pytest.mark.parametrize("d,B", [(1, 0.7), (3, 2.0), (10, 200.0), (16, 1000.0)])
def test_kernel_sinc_dB_matches_oracle(q, d, B):
    """QTT of dw/dB at eps 1e-8 against the exact derivative (the Gram-based
    sweep resolves singular values down to ~1e-8 of the norm)."""
    print(f"kernel_dB d={d} B={B}", flush=True)
    w = q.kernel_sinc_dB(d, B, 1e-8, torch.float64, DEV)
    got = q.full(w).cpu().numpy()
    assert rel(got, grads.generator_dB(d, B)) <= 3e-8


def _problem(d, seed=5, B=220.0, R=6, eps=1e-4):
    noisy, clean = G.gaussian_bumps_1d(d, seed=seed)
    cores = tt.tt_svd(noisy, eps, R)
    target = conv.toeplitz_apply_fft(clean, conv.toeplitz_generator(d, 200.0))
    return cores, target, B


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("d", [1, 6, 10, 14])
def test_conv_full_backward_matches_oracle(q, d, dt):
    """Generator and derivative QTTs from the oracle on both sides: the
    backward must reproduce the oracle's gradients of the same loss."""
    print(f"backward d={d} {dt}", flush=True)
    cores, target, B = _problem(d)
    wc, wv = oracle_qtt(conv.toeplitz_generator(d, B), 1e-10)
    bc, bv = oracle_qtt(grads.generator_dB(d, B), 1e-10)
    L, gc, gB, gw, gf = grads.grads(cores, B, target, w=wv, dw=bv)
    f = q.from_cores(cores, dt, DEV)
    w = q.from_cores(wc, dt, DEV)
    wdb = q.from_cores(bc, dt, DEV)
    y = q.toeplitz_apply(w, q.full(f))
    r = y.double() - torch.tensor(target, device=DEV)
    assert float((r * r).sum()) == pytest.approx(L, rel=1e-10 if dt == torch.float64 else 1e-5)
    gy = (2.0 * r).to(dt)
    gr, gw_t, gb = q.conv_full_backward(f, w, wdb, gy, grad_w=True)
    tol = 1e-10 if dt == torch.float64 else 2e-5
    got = gr.core_list()
    for k in range(d):
        assert rel(got[k], gc[k]) <= tol, k
    # kernel cores: the adjoint of Full of W applied to dL/dw
    gW = grads.full_adjoint(wc, gw)
    assert gw_t.ranks_host() == w.ranks_host()
    gotw = gw_t.core_list()
    for k in range(d + 1):
        assert rel(gotw[k], gW[k]) <= tol, ("W", k)
    # dL/dB = <gy, T(dw) f>: compare on the scale of its terms
    scale = float(np.linalg.norm(2.0 * (conv.toeplitz_apply_fft(tt.tt_full(cores), wv) - target))
                  * np.linalg.norm(conv.toeplitz_apply_fft(tt.tt_full(cores), bv)))
    assert abs(float(gb.cpu()) - gB) <= tol * scale


def test_autograd_function_matches_oracle(q):
    """End to end: the Function builds w(B) and dw/dB on the GPU (eps 1e-9),
    so the comparison with the exact-generator oracle is at that level."""
    d = 8
    cores, target, B = _problem(d)
    L, gc, gB, gw, gf = grads.grads(cores, B, target)
    f = q.from_cores(cores, torch.float64, DEV)
    w = q.kernel_sinc(d, B, 1e-9, torch.float64, DEV).compact()
    cparam = f.cores.clone().requires_grad_(True)
    wparam = w.cores.clone().requires_grad_(True)
    Bt = torch.tensor([B], dtype=torch.float64, requires_grad=True)
    y = q.conv_full(f, Bt, cparam, eps_dB=1e-9, w=w, wcores=wparam)
    loss = ((y - torch.tensor(target, device=DEV)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-7)
    # kernel cores against the oracle on the GPU's own generator QTT
    Wh = w.core_list()
    _, _, _, gw, _ = grads.grads(cores, B, target, w=tt.tt_full(Wh))
    gW = grads.full_adjoint(Wh, gw)
    wflat = wparam.grad.detach().cpu().numpy()
    off = 0
    for k in range(d + 1):
        n = Wh[k].size
        assert rel(wflat[off:off + n].reshape(Wh[k].shape), gW[k]) <= 1e-10, ("W", k)
        off += n
    # the gradient array has f's capacity layout; compare core by core
    flat = cparam.grad.detach().cpu().numpy()
    off = 0
    caps = f.cap
    for k in range(d):
        r0, r1 = cores[k].shape[0], cores[k].shape[2]
        blk = flat[off:off + r0 * 2 * r1].reshape(r0, 2, r1)
        assert rel(blk, gc[k]) <= 1e-7, k
        off += caps[k] * 2 * caps[k + 1]
    assert float(Bt.grad) == pytest.approx(gB, rel=1e-6)


def test_backward_at_d20_fp64(q):
    """Full-size single-signal case (d = 20, ranks <= 32, generator QTTs from
    the oracle at 1e-7): core gradients and dL/dB against the FP64 oracle of
    the same loss, and <dL/dF_k, F_k> = <dL/df, f> for every k (Full is
    linear in each core)."""
    d = 20
    print("backward d=20 f64", flush=True)
    noisy, clean = G.scatterers_1d(d, seed=2)
    cores = tt.tt_svd(noisy, 1e-4, 32)
    target = conv.toeplitz_apply_fft(clean, conv.toeplitz_generator(d, 2000.0))
    B = 2100.0
    wc, wv = oracle_qtt(conv.toeplitz_generator(d, B), 1e-7)
    bc, bv = oracle_qtt(grads.generator_dB(d, B), 1e-7)
    L, gc, gB, gw, gf = grads.grads(cores, B, target, w=wv, dw=bv)
    dt = torch.float64
    f = q.from_cores(cores, dt, DEV)
    w = q.from_cores(wc, dt, DEV)
    wdb = q.from_cores(bc, dt, DEV)
    y = q.toeplitz_apply(w, q.full(f))
    gy = 2.0 * (y - torch.tensor(target, device=DEV))
    gr, gw_t, gb = q.conv_full_backward(f, w, wdb, gy, grad_w=True)
    tol = 1e-10
    got = gr.core_list()
    fgf = float(np.dot(gf, tt.tt_full(cores)))
    for k in range(d):
        assert rel(got[k], gc[k]) <= tol, k
        assert float(np.sum(got[k] * cores[k])) == pytest.approx(fgf, rel=10 * tol)
    # kernel cores, and <dL/dW_k, W_k> = <dL/dw, w> for every k (Full of W is
    # linear in each core)
    gW = grads.full_adjoint(wc, gw)
    gotw = gw_t.core_list()
    wgw = float(np.dot(gw, wv))
    for k in range(d + 1):
        assert rel(gotw[k], gW[k]) <= tol, ("W", k)
        assert float(np.sum(gotw[k] * wc[k])) == pytest.approx(wgw, rel=10 * tol)
    scale = float(np.linalg.norm(2.0 * (conv.toeplitz_apply_fft(tt.tt_full(cores), wv) - target))
                  * np.linalg.norm(conv.toeplitz_apply_fft(tt.tt_full(cores), bv)))
    assert abs(float(gb.cpu()) - gB) <= tol * scale


def _f32(cores):
    return [np.asarray(c, dtype=np.float32).astype(np.float64) for c in cores]


def test_backward_at_d20_fp32(q):
    """d = 20 in FP32 storage: the backward is linear in the upstream gradient,
    so it is checked for one FP32 upstream gradient and FP32-rounded cores
    against the FP64 oracle on exactly those values (the residual of a loss
    near its minimum would mostly measure the rounding of the inputs)."""
    d = 20
    print("backward d=20 f32", flush=True)
    noisy, clean = G.scatterers_1d(d, seed=2)
    cores = _f32(tt.tt_svd(noisy, 1e-4, 32))
    B = 2100.0
    wc = _f32(tt.tt_svd(conv.toeplitz_generator(d, B), 1e-7))
    bc = _f32(tt.tt_svd(grads.generator_dB(d, B), 1e-7))
    wv, bv = tt.tt_full(wc), tt.tt_full(bc)
    rng = np.random.default_rng(20)
    gy = rng.standard_normal(1 << d).astype(np.float32).astype(np.float64)
    fv = tt.tt_full(cores)
    gf = conv.toeplitz_transpose_apply(gy, wv)
    gc = grads.full_adjoint(cores, gf)
    zb = conv.toeplitz_apply_fft(fv, bv)
    gB = float(gy @ zb)
    dt = torch.float32
    f = q.from_cores(cores, dt, DEV)
    w = q.from_cores(wc, dt, DEV)
    wdb = q.from_cores(bc, dt, DEV)
    gr, gw_t, gb = q.conv_full_backward(f, w, wdb, torch.tensor(gy, dtype=dt, device=DEV),
                                        grad_w=True)
    got = gr.core_list()
    for k in range(d):
        assert rel(got[k], gc[k]) <= 1e-5, k
    # dL/dw_u = sum_j gy_j f_{j+N-u} (the oracle's correlation), then Full's adjoint
    m = 4 * fv.size
    cc = np.fft.irfft(np.fft.rfft(gy, m) * np.conj(np.fft.rfft(fv, m)), m)
    gwv = np.zeros(2 * fv.size)
    u = np.arange(1, 2 * fv.size)
    gwv[1:] = cc[(u - fv.size) % m]
    gW = grads.full_adjoint(wc, gwv)
    gotw = gw_t.core_list()
    for k in range(d + 1):
        assert rel(gotw[k], gW[k]) <= 1e-5, ("W", k)
    assert abs(float(gb.cpu()) - gB) <= 1e-5 * float(np.linalg.norm(gy) * np.linalg.norm(zb))


def test_differentiation_workload_d22_fp32(q):
    """The differentiation workload at full size: d = 22, FP32 storage, signal
    cores from the decomposition of the noisy Gaussian-bump signal (eps 1e-4,
    ranks <= 32), kernel QTT at B = 220 (compacted to its ranks), target the
    convolution of the clean signal at B = 200.  Loss, every signal-core and
    kernel-core gradient and dL/dB through the autograd Function, against the
    FP64 oracle gradients of the same loss on the same (FP32-valued) cores,
    within max(2 eps, 1e-5)."""
    d, B0, Bt_, eps, R = 22, 220.0, 200.0, 1e-4, 32
    print("case: differentiation d=22 f32", flush=True)
    dt = torch.float32
    noisy, clean = G.diff_workload(d)
    target = conv.toeplitz_apply_fft(clean, conv.toeplitz_generator(d, Bt_))
    f = q.decompose(torch.tensor(noisy, dtype=dt, device=DEV), eps, R)
    w = q.kernel_sinc(d, B0, eps / 10, dt, DEV).compact()
    cparam = f.cores.clone().requires_grad_(True)
    wparam = w.cores.clone().requires_grad_(True)
    Bt = torch.tensor([B0], dtype=torch.float64, requires_grad=True)
    y = q.conv_full(f, Bt, cparam, eps_dB=1e-7, w=w, wcores=wparam)
    loss = ((y.double() - torch.tensor(target, device=DEV)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    Fh, Wh = f.core_list(), w.core_list()
    Dh = q.kernel_sinc_dB(d, B0, 1e-7, dt, DEV).core_list()
    L, gc, gB, gw, _ = grads.grads(Fh, B0, target, w=tt.tt_full(Wh), dw=tt.tt_full(Dh))
    gW = grads.full_adjoint(Wh, gw)
    tol = max(2 * eps, 1e-5)
    eL = abs(float(loss.detach()) - L) / L
    cflat = cparam.grad.detach().cpu().double().numpy()
    wflat = wparam.grad.detach().cpu().double().numpy()
    ef, off = [], 0
    for k in range(d):
        n = Fh[k].size
        ef.append(rel(cflat[off:off + n].reshape(Fh[k].shape), gc[k]))
        off += f.cap[k] * 2 * f.cap[k + 1]
    ew, off = [], 0
    for k in range(d + 1):
        n = Wh[k].size
        ew.append(rel(wflat[off:off + n].reshape(Wh[k].shape), gW[k]))
        off += n
    eB = abs(float(Bt.grad) - gB) / abs(gB)
    print(f"d=22 f32: loss {eL:.2e}, signal cores max {max(ef):.2e}, kernel cores max "
          f"{max(ew):.2e}, dL/dB {eB:.2e} (W ranks {w.ranks_host()})", flush=True)
    assert eL <= tol
    assert max(ef) <= tol and max(ew) <= tol and eB <= tol


def test_backward_rejects_bad_arguments(q):
    f = q.from_cores(tt.tt_svd(np.arange(16.0), 0.0), torch.float64, DEV)
    w = q.kernel_sinc(4, 3.0, 1e-10, torch.float64, DEV)
    with pytest.raises(q.QttError):
        q.conv_full_backward(f, w, None, torch.zeros(8, dtype=torch.float64, device=DEV))
    with pytest.raises(q.QttError):
        q.toeplitz_apply(w, torch.zeros(16, dtype=torch.float32, device=DEV))
