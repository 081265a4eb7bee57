"""GPU parity: every C-ABI call against the FP64 CPU oracle on seeded inputs.

Tolerances (relative L2 of full arrays): 1e-10 for the FP64 path,
max(2 eps, 1e-5) for FP32 storage; ranks exact.  The FP32 path is compared
with the oracle run on the same FP32-rounded input.
"""

import math
import sys

import numpy as np
import pytest

from oracle import conv, pipeline, tt
from synthetic import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_13339_amd as q  # noqa: E402

DEV = "cuda"


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def tol_for(dt, eps):
    return 1e-10 if dt == torch.float64 else max(2 * eps, 1e-5)


def announce(*a):
    print("case:", *a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------- full

@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 12, 16])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_full_random_cores(d, dt):
    announce("full", d, dt)
    rng = np.random.default_rng(100 + d)
    ranks = [1] + [int(rng.integers(1, 7)) for _ in range(d - 1)] + [1]
    cores = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) for k in range(d)]
    if dt == torch.float32:
        cores = [c.astype(np.float32).astype(np.float64) for c in cores]
    out = q.full(q.from_cores(cores, dt, DEV)).cpu().numpy()
    assert rel(out, tt.tt_full(cores)) <= (1e-13 if dt == torch.float64 else 1e-5)


# -------------------------------------------------------------- decompose

DECOMP_CASES = [
    ("random_d2", lambda: np.random.default_rng(1).standard_normal(4), 0.0, 0),
    ("random_d6", lambda: np.random.default_rng(2).standard_normal(64), 1e-2, 0),
    ("bumps_d12", lambda: G.gaussian_bumps_1d(12, 1)[0], 1e-3, 0),
    ("scatter_d13_R32", lambda: G.scatterers_1d(13, 2)[0], 1e-4, 32),
    ("scatter_d14_R32", lambda: G.scatterers_1d(14, 2)[0], 1e-4, 32),
    ("scatter_d16_R32", lambda: G.scatterers_1d(16, 2)[0], 1e-4, 32),
    ("scatter_d16_R5", lambda: G.scatterers_1d(16, 2)[0], 1e-4, 5),
    ("scatter_d20_R32_e4", lambda: G.scatterers_1d(20, 2)[0], 1e-4, 32),
    ("scatter_d20_R32_e2", lambda: G.scatterers_1d(20, 2)[0], 1e-2, 32),
    # cap 48: unfoldings of 96 rows use the global-memory eigensolver path
    ("scatter_d17_R48", lambda: G.scatterers_1d(17, 2)[0], 1e-4, 48),
    # caps 20 and 24: Grams of order 40 and 48 (Sturm counts padded to 48
    # rows) and orders 10..16 (the four-rows-per-lane reduction)
    ("scatter_d14_R20", lambda: G.scatterers_1d(14, 2)[0], 1e-4, 20),
    ("scatter_d15_R24", lambda: G.scatterers_1d(15, 5)[0], 1e-4, 24),
    ("scatter_d13_R6", lambda: G.scatterers_1d(13, 7)[0], 1e-4, 6),
]


@pytest.mark.parametrize("name,gen,eps,R", DECOMP_CASES, ids=[c[0] for c in DECOMP_CASES])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_decompose_matches_ttsvd(name, gen, eps, R, dt):
    announce("decompose", name, dt)
    x = gen()
    if dt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    ref, info = tt.tt_svd(x, eps, R, return_info=True)
    t, sv = q.decompose(torch.tensor(x, dtype=dt, device=DEV), eps, R, return_sv=True)
    out = q.full(t).cpu().numpy()
    ranks = t.ranks_host()
    if info["margin"] > 1e-5 or dt == torch.float64:
        assert ranks == info["ranks"]
    assert t.status_host() == 0
    assert rel(out, tt.tt_full(ref)) <= tol_for(dt, eps)
    if dt == torch.float64:
        # squared singular values (Gram eigenvalues) to 1e-12 of the largest
        svh = sv.cpu().numpy()
        s0 = max(s[0] for s in info["sv"])
        for k, s in enumerate(info["sv"]):
            assert np.max(np.abs(svh[k][: len(s)] ** 2 - s * s)) <= 1e-12 * s0 * s0, k
    # left-orthonormal cores (all but the last)
    for c in t.core_list()[:-1]:
        U = c.reshape(-1, c.shape[2], order="F")
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= (1e-10 if dt == torch.float64
                                                                   else 1e-5)


# Without the singular-value output and with a binding cap the eigensolver
# computes only the cap largest eigenvalues and takes the rank rule's tail
# sums from the trace: same ranks, cores and reconstruction as the oracle.
@pytest.mark.parametrize("name,d,seed,eps,R", [("scatter_d20_R32", 20, 2, 1e-4, 32),
                                               ("scatter_d16_R16", 16, 3, 1e-4, 16),
                                               ("scatter_d14_R8", 14, 4, 1e-3, 8)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_decompose_capped_without_sv(name, d, seed, eps, R, dt):
    announce("decompose top-cap", name, dt)
    x = G.scatterers_1d(d, seed)[0]
    if dt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    ref, info = tt.tt_svd(x, eps, R, return_info=True)
    t = q.decompose(torch.tensor(x, dtype=dt, device=DEV), eps, R)
    ranks = t.ranks_host()
    if info["margin"] > 1e-5 or dt == torch.float64:
        assert ranks == info["ranks"]
    assert max(ranks) == R  # the cap binds
    assert rel(q.full(t).cpu().numpy(), tt.tt_full(ref)) <= tol_for(dt, eps)
    for c in t.core_list()[:-1]:
        U = c.reshape(-1, c.shape[2], order="F")
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= (1e-10 if dt == torch.float64
                                                                   else 1e-5)


def _padded(v, K):
    out = np.zeros(1 << K)
    out[: v.size] = v
    return out


def _lowrank_noise(d, seed, noise):
    """Three smooth terms (QTT ranks <= 5) plus white noise of the given std."""
    x = np.arange(1 << d) / float(1 << d)
    rng = np.random.default_rng(seed)
    v = np.sin(2 * np.pi * 5 * x + 0.3) + 0.8 * np.exp(-3 * x) + 0.3 * np.cos(2 * np.pi * 11 * x)
    return v + noise * rng.standard_normal(v.size)


def _sinusoids(d, seed, n=12):
    """n cosines spread up to 0.46 N cycles: every unfolding of QTT level k
    (rows = the low k index bits) has rank min(2^k, 2n), well conditioned."""
    N = 1 << d
    t = np.arange(N) / float(N)
    rng = np.random.default_rng(seed)
    return sum(np.cos(2 * np.pi * round(N * (j + 0.37) / (2 * n + 3)) * t + rng.uniform(0, 2 * np.pi))
               for j in range(1, n + 1))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_decompose_level_full_rank_then_deficient(dt):
    """Level steps without the singular-value output: steps 1-4 keep full rank
    (their positive-definiteness tests pass and they keep V = I), step 5 has
    rank 24 of 32 with no cap (its test fails on a pivot, and it and every
    later step take the eigensolver): same ranks and tensor as the oracle,
    left-orthonormal cores."""
    announce("decompose level full rank then deficient", dt)
    x = _sinusoids(16, 11)
    if dt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    eps, R = 1e-6, 0
    ref, info = tt.tt_svd(x, eps, R, return_info=True)
    assert info["ranks"][:7] == [1, 2, 4, 8, 16, 24, 24] and info["margin"] > 0.5
    t = q.decompose(torch.tensor(x, dtype=dt, device=DEV), eps, R)
    assert t.ranks_host() == info["ranks"]
    assert t.status_host() == 0
    assert rel(q.full(t).cpu().numpy(), tt.tt_full(ref)) <= tol_for(dt, eps)
    for c in t.core_list()[:-1]:
        U = c.reshape(-1, c.shape[2], order="F")
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= (1e-10 if dt == torch.float64
                                                                   else 1e-5)


# Modification (3) of Section 5: the singular-value drop-off cut, alone
# (eps = 0) or with the tolerance and the cap.  The cases cut at several
# unfoldings (to rank 1 where the two sample halves are nearly equal) and run
# through the tail-only, level + eig-step and tail paths.
DROP_CASES = [
    ("ex1_K12_d02", lambda: _padded(G.paper_example1(12, 0, True)[0], 12), 0.0, 32, 0.02),
    ("ex1_K20_d02", lambda: _padded(G.paper_example1(20, 0, True)[0], 20), 0.0, 32, 0.02),
    ("ex2_K16_d01", lambda: _padded(G.paper_example2(16, 0)[0], 16), 0.0, 32, 0.01),
    ("lowrank_d10_d01", lambda: _lowrank_noise(10, 10, 1e-5), 0.0, 0, 0.01),
    ("lowrank_d16_e6_d05", lambda: _lowrank_noise(16, 16, 1e-4), 1e-6, 32, 0.05),
    ("lowrank_d20_d01", lambda: _lowrank_noise(20, 20, 1e-5), 0.0, 32, 0.01),
]


@pytest.mark.parametrize("name,gen,eps,R,delta", DROP_CASES, ids=[c[0] for c in DROP_CASES])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_decompose_dropoff_matches_oracle(name, gen, eps, R, delta, dt):
    announce("decompose drop-off", name, dt)
    x = gen()
    if dt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    ref, info = tt.tt_svd(x, eps, R, return_info=True, delta=delta)
    t = q.decompose(torch.tensor(x, dtype=dt, device=DEV), eps, R, delta=delta)
    ranks = t.ranks_host()
    # every decision of the cases is at least 1e-4 (relative) from its threshold
    assert info["delta_margin"] > 1e-4 and info["margin"] > 1e-4
    assert ranks == info["ranks"]
    assert t.status_host() == 0
    assert rel(q.full(t).cpu().numpy(), tt.tt_full(ref)) <= tol_for(dt, 1e-5)
    # with eps = 0 the drop-off keeps singular values down to the drop (1e-3
    # of the largest here), and cores formed on the short side of an
    # unfolding (u = X^T v / sigma) are orthonormal only to the Gram route's
    # floor u (sigma_1 / sigma_r)^2, u the FP64 unit roundoff
    floor = max(1.1e-16 * (sk[0] / sk[r - 1]) ** 2
                for sk, r in zip(info["sv"], info["ranks"][1:]) if sk[0] > 0)
    otol = max(1e-10, 10 * floor) if dt == torch.float64 else 1e-5
    for c in t.core_list()[:-1]:
        U = c.reshape(-1, c.shape[2], order="F")
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= otol


def test_decompose_dropoff_zero_and_off():
    """A zero vector has no drop (0/0) and rank 1 everywhere; delta = 0 is qtt_decompose."""
    announce("decompose drop-off zero/off")
    t = q.decompose(torch.zeros(1 << 12, dtype=torch.float64, device=DEV), 0.0, 0, delta=0.5)
    assert t.ranks_host() == [1] * 13 and t.status_host() == 0
    assert not np.any(q.full(t).cpu().numpy())
    x = torch.tensor(G.scatterers_1d(14, 2)[0], dtype=torch.float64, device=DEV)
    a = q.decompose(x, 1e-4, 32)
    b = q.decompose(x, 1e-4, 32, delta=0.0)
    assert a.ranks_host() == b.ranks_host()
    assert torch.equal(q.full(a), q.full(b))


@pytest.mark.parametrize("kind,param", [("exp", 3.0), ("sin", 5.0), ("cos", 2.0), ("poly", 1),
                                        ("poly", 3)])
@pytest.mark.parametrize("d", [10, 16])
def test_decompose_closed_forms(kind, param, d):
    announce("closed form", kind, param, d)
    x = G.closed_form_signal(kind, d, param)
    eps = 1e-6
    ref, info = tt.tt_svd(x, eps, return_info=True)
    t = q.decompose(torch.tensor(x, dtype=torch.float64, device=DEV), eps)
    assert t.ranks_host() == info["ranks"]
    expect = {"exp": 1, "sin": 2, "cos": 2}.get(kind, int(param) + 1)
    assert max(t.ranks_host()) == expect
    assert rel(q.full(t).cpu().numpy(), x) <= 1e-6


@pytest.mark.parametrize("kind,d,dt", [("exp", 28, torch.float64), ("sin", 27, torch.float64),
                                        ("exp", 28, torch.float32)])
def test_decompose_large_closed_form(kind, d, dt):
    """Largest sizes (2^27..2^28 samples, up to 2 GiB): the samples are made on the
    device, the ranks are the closed-form ones (1 for exp, at most 2 for sin) and
    sampled entries, each a product of core slices on the host, match the function
    (sin: within the error bound of Algorithm 1)."""
    announce("large closed form", kind, d, dt)
    n = 1 << d
    xs = torch.arange(n, device=DEV, dtype=torch.float64) / n
    x = torch.exp(0.7 * xs) if kind == "exp" else torch.sin(2 * math.pi * 3 * xs + 0.3)
    x = x.to(dt)
    del xs
    # Gram sums over 2^28 samples resolve singular values only down to about
    # sqrt(u n) of the norm, so the tolerance stays well above that floor
    eps = 1e-4
    t = q.decompose(x, eps)
    ranks = t.ranks_host()
    assert t.status_host() == 0
    cores = t.core_list()
    idx = np.random.default_rng(d).integers(0, n, 2000)
    xh = x[torch.tensor(idx, device=DEV)].double().cpu().numpy()
    got = np.array([tt.tt_entry(cores, int(i)) for i in idx])
    if kind == "exp":
        # rank 1 at every unfolding: only rounding is discarded
        assert max(ranks) == 1
        tol = 1e-10 if dt == torch.float64 else 2e-5
        assert np.max(np.abs(got - xh)) <= tol * np.max(np.abs(xh))
    else:
        # rank <= 2; at the finest bits sigma_2 / sigma_1 falls below eps and the
        # rule keeps rank 1, within the bound ||x - x_TT|| <= eps ||x|| (here on
        # the RMS of the sampled entries)
        assert max(ranks) == 2
        rms_err = float(np.sqrt(np.mean((got - xh) ** 2)))
        assert rms_err <= 1.5 * eps * float(np.sqrt(np.mean(xh ** 2)))
    del x


def test_decompose_zero_vector():
    announce("zero vector")
    t = q.decompose(torch.zeros(1 << 15, dtype=torch.float64, device=DEV), 1e-3)
    assert t.ranks_host() == [1] * 16
    assert float(q.full(t).abs().max()) == 0.0


@pytest.mark.parametrize("d", [8, 16])
def test_decompose_nonfinite_sets_status(d):
    announce("nonfinite", d)
    x = torch.ones(1 << d, dtype=torch.float64, device=DEV)
    x[7] = float("nan")
    t = q.decompose(x, 1e-3)
    torch.cuda.synchronize()
    assert t.status_host() & q.QTT_STATUS_NONFINITE


def test_decompose_rank_capacity_flag():
    """Uncapped white noise at d=16 has eps-ranks above the 64 capacity."""
    announce("rankcap flag")
    x = np.random.default_rng(5).standard_normal(1 << 16)
    t = q.decompose(torch.tensor(x, device=DEV), 1e-6)
    assert t.status_host() & q.QTT_STATUS_RANKCAP
    assert max(t.ranks_host()) == q.QTT_MAX_RANK


# ------------------------------------------------------------------ kernel

@pytest.mark.parametrize("d,B,ew", [(1, 1.0, 1e-5), (4, 3.0, 1e-5), (12, 200.0, 1e-4),
                                    (16, 500.0, 1e-5), (20, 2000.0, 1e-5)])
def test_kernel_sinc_matches_oracle(d, B, ew):
    announce("kernel", d, B)
    w = conv.toeplitz_generator(d, B)
    ref, info = tt.tt_svd(w, ew, return_info=True)
    W = q.kernel_sinc(d, B, ew, torch.float64, DEV)
    assert W.ranks_host() == info["ranks"]
    assert rel(q.full(W).cpu().numpy(), tt.tt_full(ref)) <= 1e-10


# -------------------------------------------------------------------- conv

@pytest.mark.parametrize("d,B,R", [(2, 1.0, 0), (4, 3.0, 0), (8, 20.0, 4), (12, 200.0, 8),
                                   (16, 500.0, 8)])
def test_conv_exact_toeplitz(d, B, R):
    announce("conv", d, B)
    x = G.gaussian_bumps_1d(d, 1)[0]
    F = tt.tt_svd(x, 1e-3, R)
    Wt = tt.tt_full(tt.tt_svd(conv.toeplitz_generator(d, B), 1e-5))
    y = q.conv(q.from_cores(F, torch.float64, DEV), [q.kernel_sinc(d, B, 1e-5, torch.float64, DEV)])
    ref = conv.toeplitz_apply(tt.tt_full(F), Wt)
    assert rel(q.full(y).cpu().numpy(), ref) <= 1e-11
    # output bond is 2 * rho_k * r_k inside, 1 at the ends
    yr = y.ranks_host()
    assert yr[0] == 1 and yr[-1] == 1


@pytest.mark.parametrize("d", [3, 5])
def test_conv_operator_columns(d):
    """Applying the QTT Toeplitz operator to unit vectors e_i returns column i of T."""
    announce("conv columns", d)
    n = 1 << d
    rng = np.random.default_rng(d)
    w = rng.standard_normal(2 * n)
    W = tt.tt_svd(w, 0.0)
    Wg = q.from_cores(W, torch.float64, DEV)
    T = conv.toeplitz_dense(tt.tt_full(W))
    for i in range(n):
        cores = [np.array([1.0 - ((i >> k) & 1), float((i >> k) & 1)]).reshape(1, 2, 1)
                 for k in range(d)]
        y = q.conv(q.from_cores(cores, torch.float64, DEV), [Wg])
        assert np.allclose(q.full(y).cpu().numpy(), T[:, i], atol=1e-12)


def test_conv_2d_separable():
    announce("conv 2d")
    dy, dx = 5, 6
    img = G.sar_image_2d(dy, dx, seed=3, n_scatterers=10)[0]
    F = tt.tt_svd(img.ravel(), 1e-3, 8)
    wx = tt.tt_full(tt.tt_svd(conv.toeplitz_generator(dx, 40.0), 1e-6))
    wy = tt.tt_full(tt.tt_svd(conv.toeplitz_generator(dy, 20.0), 1e-6))
    y = q.conv(q.from_cores(F, torch.float64, DEV),
               [q.kernel_sinc(dx, 40.0, 1e-6), q.kernel_sinc(dy, 20.0, 1e-6)], [dx, dy])
    ref = conv.toeplitz_apply_2d(tt.tt_full(F).reshape(1 << dy, 1 << dx), wy, wx, fft=False)
    assert rel(q.full(y).cpu().numpy(), ref) <= 1e-11


# ------------------------------------------------------------------- round

@pytest.mark.parametrize("d,B,eps", [(10, 50.0, 1e-3), (14, 300.0, 1e-4), (16, 500.0, 1e-2)])
def test_round_equals_ttsvd_of_represented_tensor(d, B, eps):
    announce("round", d, B, eps)
    x = G.scatterers_1d(d, 2)[0]
    f = q.decompose(torch.tensor(x, device=DEV), eps, 16)
    y = q.conv(f, [q.kernel_sinc(d, B, eps / 10)])
    yfull = q.full(y).cpu().numpy()
    ref, info = tt.tt_svd(yfull, eps, return_info=True)
    z = q.round(y, eps)
    assert z.ranks_host() == info["ranks"]
    assert rel(q.full(z).cpu().numpy(), tt.tt_full(ref)) <= 1e-10


# ---------------------------------------------------------------- pipeline

PIPE_CASES = [
    ("line_d12", 12, "bumps", 200.0, 1e-3, 0),
    ("line_d16", 16, "scatter", 500.0, 1e-4, 32),
    ("line_d20_e4", 20, "scatter", 2000.0, 1e-4, 32),
    ("line_d20_e2", 20, "scatter", 2000.0, 1e-2, 32),
]


@pytest.mark.parametrize("name,d,kind,B,eps,R", PIPE_CASES, ids=[c[0] for c in PIPE_CASES])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_pipeline_matches_oracle(name, d, kind, B, eps, R, dt):
    announce("pipeline", name, dt)
    x = G.gaussian_bumps_1d(d, 1)[0] if kind == "bumps" else G.scatterers_1d(d, 2)[0]
    if dt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    ref = pipeline.pipeline_1d(x, B, eps, R)
    out, st = q.pipeline(torch.tensor(x, dtype=dt, device=DEV), B, eps, R)
    assert rel(out.cpu().numpy(), ref["out"]) <= tol_for(dt, eps)
    if dt == torch.float64 or ref["Z_info"]["margin"] > 1e-5:
        assert st["z"].ranks_host() == ref["Z_ranks"]
        assert st["f"].ranks_host() == ref["F_ranks"]


def test_pipeline_image_small():
    announce("pipeline image")
    img = G.sar_image_2d(6, 7, seed=3, n_scatterers=12)[0]
    ref = pipeline.pipeline_2d(img, 40.0, 30.0, 1e-3, 8, fft=False)
    out, st = q.pipeline(torch.tensor(img, device=DEV), (40.0, 30.0), 1e-3, 8,
                         shape2d=img.shape)
    assert rel(out.cpu().numpy(), ref["out"]) <= 1e-10
    assert st["z"].ranks_host() == ref["Z_ranks"]


def test_pipeline_repeatable():
    """Same input twice gives bitwise identical output (fixed reduction order)."""
    announce("repeatable")
    x = torch.tensor(G.scatterers_1d(16, 2)[0], device=DEV)
    a, _ = q.pipeline(x, 500.0, 1e-4, 32)
    b, _ = q.pipeline(x, 500.0, 1e-4, 32)
    assert torch.equal(a, b)


def test_pipeline_graph_replays():
    """The pipeline captured into a graph: every replay equals the eager result bitwise,
    with eager pipelines between the replays, and new samples copied into the captured
    input are picked up."""
    announce("pipeline graph")
    x = torch.tensor(G.scatterers_1d(16, 2)[0], device=DEV)
    ref, _ = q.pipeline(x, 500.0, 1e-4, 32)
    pg = q.PipelineGraph(x, 500.0, 1e-4, 32)
    for _ in range(3):
        out = pg.run()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        q.pipeline(x, 500.0, 1e-4, 32)
        torch.cuda.synchronize()
    x2 = torch.tensor(G.scatterers_1d(16, 7)[0], device=DEV)
    ref2, st2 = q.pipeline(x2, 500.0, 1e-4, 32)
    x.copy_(x2)
    out = pg.run()
    torch.cuda.synchronize()
    assert torch.equal(out, ref2)
    assert pg.stages["z"].ranks_host() == st2["z"].ranks_host()


# ------------------------------------------------------------- error paths

def test_binding_raises_on_bad_arguments():
    announce("errors")
    x = torch.ones(7, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        q.decompose(x, 1e-3)
    y = torch.ones(16, dtype=torch.float64, device=DEV)
    with pytest.raises(q.QttError):
        q.decompose(y, -1.0)
    with pytest.raises(q.QttError):
        q.decompose(y, 1e-3, -2)
