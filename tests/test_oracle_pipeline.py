"""Pins of the composed oracle pipeline and its gradients."""

import numpy as np
import pytest

from oracle import conv, grads, pipeline, tt
from synthetic import generators as G


def test_pipeline_line_d12_composition_and_denoising():
    noisy, clean = G.gaussian_bumps_1d(12, seed=1)
    res = pipeline.pipeline_1d(noisy, 200.0, 1e-3)
    # the composition is what the docstring states
    f_t = tt.tt_full(tt.tt_svd(noisy, 1e-3))
    w_t = tt.tt_full(tt.tt_svd(conv.toeplitz_generator(12, 200.0), 1e-4))
    y = conv.toeplitz_apply(f_t, w_t)
    assert np.allclose(res["y"], y, rtol=0, atol=1e-14 * np.max(np.abs(y)))
    z = tt.tt_full(tt.tt_svd(y, 1e-3))
    assert np.allclose(res["out"], z, rtol=0, atol=1e-13 * np.max(np.abs(z)))
    # rounding an exact TT of y gives the same tensor
    zr = tt.tt_full(tt.tt_round(tt.tt_svd(y, 0.0), 1e-3))
    assert np.linalg.norm(zr - z) <= 1e-11 * np.linalg.norm(z)
    ref = pipeline.clean_reference_1d(clean, 200.0)
    e_out = pipeline.relative_error(res["out"], ref)
    e_noisy = pipeline.relative_error(pipeline.clean_reference_1d(noisy, 200.0), ref)
    assert e_out < e_noisy * 1.05
    assert res["Z_ranks"][0] == 1 and res["Z_ranks"][-1] == 1


def test_pipeline_rank_cap_denoises():
    """Section 6 / Table 7.1: max-rank truncation removes most of the noise on Example 1."""
    K = 16
    noisy, clean, _, _ = G.paper_example1(K, 0, full_grid=True)
    B = (1 << K) / 4.0                         # resolution 4 dx as in Example 1
    ref = pipeline.clean_reference_1d(clean, B)
    e_noisy = pipeline.relative_error(pipeline.clean_reference_1d(noisy, B), ref)
    capped = pipeline.pipeline_1d(noisy, B, 1e-4, max_rank=10)
    assert max(capped["F_ranks"]) == 10
    assert pipeline.relative_error(capped["out"], ref) < 0.5 * e_noisy


def test_pipeline_2d_separable():
    noisy, clean = G.sar_image_2d(5, 6, seed=3, n_scatterers=10)
    res = pipeline.pipeline_2d(noisy, 40.0, 20.0, 1e-3, fft=False)
    f_t = tt.tt_full(res["F"]).reshape(noisy.shape)
    gx, dx = conv.sinc_kernel_samples(6, 40.0)
    gy, dy = conv.sinc_kernel_samples(5, 20.0)
    # with an exact (eps_w = 0) kernel the 2-D Toeplitz product equals (2.2) with D = 2
    exact_w = pipeline.pipeline_2d(noisy, 40.0, 20.0, 1e-3, eps_w=0.0, fft=False)
    ref = conv.conv_same_2d(f_t, gy, gx, dy, dx)
    assert np.allclose(exact_w["y"], ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    assert res["out"].shape == noisy.shape


def test_pipeline_2d_dropoff_composition():
    """The drop-off cut (modification (3) of Section 5) in the 2-D pipeline acts on
    the data decomposition and on the rounding, as in the 1-D pipeline."""
    _, clean, _, _ = G.paper_example3(7)
    noisy = np.zeros((64, 64))
    noisy[:63, :63] = clean
    delta = 0.05
    res = pipeline.pipeline_2d(noisy, 12.0, 12.0, 0.0, max_rank=64, round_max_rank=64,
                               fft=False, delta=delta)
    _, finfo = tt.tt_svd(noisy.ravel(), 0.0, 64, return_info=True, delta=delta)
    assert res["F_ranks"] == finfo["ranks"]
    _, zinfo = tt.tt_svd(res["y"].ravel(), 0.0, 64, return_info=True, delta=delta)
    assert res["Z_ranks"] == zinfo["ranks"]
    plain = pipeline.pipeline_2d(noisy, 12.0, 12.0, 0.0, max_rank=64, round_max_rank=64,
                                 fft=False)
    assert all(a <= b for a, b in zip(res["F_ranks"], plain["F_ranks"]))
    assert sum(res["F_ranks"]) < sum(plain["F_ranks"])


def test_kernel_core_gradients_central_differences_d10():
    """dL/dW_k for the kernel cores W (d + 1 modes) of L = ||T(full(W)) full(F) - t||^2:
    the adjoint of Full applied to dL/dw, against central differences (h = 1e-6)."""
    d = 10
    noisy, clean = G.gaussian_bumps_1d(d, seed=6)
    F = tt.tt_svd(noisy, 1e-4, 6)
    W = tt.tt_svd(conv.toeplitz_generator(d, 220.0), 1e-6)
    target = conv.toeplitz_apply(clean, conv.toeplitz_generator(d, 200.0))
    _, _, _, gw, _ = grads.grads(F, 220.0, target, w=tt.tt_full(W))
    gW = grads.full_adjoint(W, gw)
    h = 1e-6
    rng = np.random.default_rng(1)

    def lossW(Wc):
        return grads.loss(F, 220.0, target, w=tt.tt_full(Wc))

    for k in (0, 4, d - 1, d):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in W[k].shape)
            c2 = [c.copy() for c in W]
            c2[k][idx] += h
            lp = lossW(c2)
            c2[k][idx] -= 2 * h
            lm = lossW(c2)
            assert gW[k][idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8)


def test_grads_central_differences_d10():
    d = 10
    noisy, clean = G.gaussian_bumps_1d(d, seed=5)
    cores = tt.tt_svd(noisy, 1e-4, 6)
    target = conv.toeplitz_apply(clean, conv.toeplitz_generator(d, 200.0))
    B = 220.0
    L, gc, gB, gw, gf = grads.grads(cores, B, target)
    h = 1e-6
    fd = (grads.loss(cores, B + h, target) - grads.loss(cores, B - h, target)) / (2 * h)
    assert gB == pytest.approx(fd, rel=1e-5, abs=1e-9)
    rng = np.random.default_rng(0)
    for k in (0, 3, d - 1):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in cores[k].shape)
            c2 = [c.copy() for c in cores]
            c2[k][idx] += h
            lp = grads.loss(c2, B, target)
            c2[k][idx] -= 2 * h
            lm = grads.loss(c2, B, target)
            assert gc[k][idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9)


def test_adjoint_dot_product():
    d = 9
    rng = np.random.default_rng(2)
    w = conv.toeplitz_generator(d, 50.0)
    f = rng.standard_normal(1 << d)
    y = rng.standard_normal(1 << d)
    lhs = conv.toeplitz_apply(f, w) @ y
    rhs = f @ conv.toeplitz_transpose_apply(y, w)
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_grad_w_definition_small():
    """dL/dw_u by brute force on a tiny case."""
    d = 4
    n = 1 << d
    rng = np.random.default_rng(9)
    cores = tt.tt_svd(rng.standard_normal(n), 0.0)
    t = rng.standard_normal(n)
    B = 3.0
    L, gc, gB, gw, gf = grads.grads(cores, B, t)
    f = tt.tt_full(cores)
    y = conv.toeplitz_apply(f, conv.toeplitz_generator(d, B))
    gy = 2 * (y - t)
    ref = np.zeros(2 * n)
    for j in range(n):
        for i in range(n):
            ref[j - i + n] += gy[j] * f[i]
    assert np.allclose(gw, ref, atol=1e-12)


def test_full_adjoint_multilinear_identity():
    """full is linear in each core, so <dG/dF_k, F_k> = G = <g, full(F)> for every k."""
    d = 8
    rng = np.random.default_rng(11)
    cores = tt.tt_svd(rng.standard_normal(1 << d), 1e-2, 5)
    g = rng.standard_normal(1 << d)
    G = float(g @ tt.tt_full(cores))
    gc = grads.full_adjoint(cores, g)
    for k in range(d):
        assert float(np.sum(gc[k] * cores[k])) == pytest.approx(G, rel=1e-12)


def test_generator_dB_central_differences():
    d, B, h = 7, 30.0, 1e-6
    fd = (conv.toeplitz_generator(d, B + h) - conv.toeplitz_generator(d, B - h)) / (2 * h)
    assert np.allclose(grads.generator_dB(d, B), fd, rtol=0, atol=1e-8)


def test_pipeline_dropoff_composition():
    """Modification (3) in the pipeline: the data decomposition and the rounding take the
    drop-off cut (their ranks are the rule applied to their own spectra), the kernel keeps
    the tolerance rule, and delta = 0 is the plain pipeline."""
    K = 12
    noisy, clean, _, _ = G.paper_example1(K, 0, full_grid=True)
    B = (1 << K) / 4.0
    res = pipeline.pipeline_1d(noisy, B, 0.0, delta=0.02)
    plain = pipeline.pipeline_1d(noisy, B, 0.0)
    assert res["W_ranks"] == plain["W_ranks"]
    for info, ranks in ((res["F_info"], res["F_ranks"]), (res["Z_info"], res["Z_ranks"])):
        for k, s in enumerate(info["sv"], start=1):
            rd = tt.dropoff_rank(s, 0.02)
            assert ranks[k] == (rd if rd is not None else tt.truncation_rank(s, 0.0, 0))
    same = pipeline.pipeline_1d(noisy, B, 1e-3, delta=0.0)
    ref = pipeline.pipeline_1d(noisy, B, 1e-3)
    assert np.array_equal(same["out"], ref["out"])
