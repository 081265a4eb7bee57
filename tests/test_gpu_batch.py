"""GPU parity of the batched form (many lines of uneven length through the
whole pipeline in a few launches / one hipGraph) against the FP64 oracle,
line by line."""

import numpy as np
import pytest
import torch

from oracle import pipeline as P
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


def _lines(ds, seed=40):
    """Noisy scatterer lines of the given lengths and bandwidths."""
    rng = np.random.default_rng(seed)
    xs, Bs = [], []
    for i, d in enumerate(ds):
        noisy, _ = G.scatterers_1d(d, seed=seed * 100 + i, n_scatterers=int(rng.integers(4, 16)))
        xs.append(noisy)
        Bs.append(float(rng.uniform(0.05, 0.4) * (1 << d)))
    return xs, Bs


# lengths cover the one-workgroup tail (N <= 8192), the level + eig-step path
# (N > 8192) and the trivial d = 1 line, in an order the tasks get re-sorted from
DS = [1, 3, 14, 6, 9, 12, 13, 15, 10, 2, 16, 11]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_batch_matches_oracle_per_line(q, dt):
    eps, R = 1e-4, 32
    xs, Bs = _lines(DS)
    print(f"batch {len(DS)} lines {dt}", flush=True)
    b = q.Batch(DS, Bs, dt, eps, R, device=DEV)
    x = torch.tensor(np.concatenate(xs), dtype=dt, device=DEV)
    out = b.run(x, graph=False)
    torch.cuda.synchronize()
    st = b.status()
    assert int(st.abs().sum()) == 0, st
    tol = 1e-10 if dt == torch.float64 else max(2 * eps, 1e-5)
    for l, (xl, Bl) in enumerate(zip(xs, Bs)):
        ref = P.pipeline_1d(xl, Bl, eps, R)
        got = b.line(out, l).double().cpu().numpy()
        assert b.ranks(l, 0) == ref["F_ranks"], (l, b.ranks(l, 0), ref["F_ranks"])
        assert b.ranks(l, 2) == ref["Z_ranks"], (l, b.ranks(l, 2), ref["Z_ranks"])
        assert rel(got, ref["out"]) <= tol, (l, DS[l], rel(got, ref["out"]))


def test_batch_graph_replay_and_new_data(q):
    eps, R = 1e-4, 32
    dt = torch.float64
    xs, Bs = _lines(DS, seed=41)
    b = q.Batch(DS, Bs, dt, eps, R, device=DEV)
    x = torch.tensor(np.concatenate(xs), dtype=dt, device=DEV)
    out0 = b.run(x, graph=False).clone()
    out = torch.empty_like(x)
    for _ in range(3):
        b.run(x, out, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out, out0)
    # new samples in the same buffer: the captured graph reads them
    xs2, _ = _lines(DS, seed=42)
    x.copy_(torch.tensor(np.concatenate(xs2), dtype=dt, device=DEV))
    b.run(x, out, graph=True)
    torch.cuda.synchronize()
    for l in (0, 2, 7, 10):
        ref = P.pipeline_1d(xs2[l], Bs[l], eps, R)
        assert rel(b.line(out, l).cpu().numpy(), ref["out"]) <= 1e-10, l


def test_batch_equals_single_line_path(q):
    eps, R = 1e-4, 32
    dt = torch.float64
    ds = [12, 15, 16]
    xs, Bs = _lines(ds, seed=43)
    b = q.Batch(ds, Bs, dt, eps, R, device=DEV)
    x = torch.tensor(np.concatenate(xs), dtype=dt, device=DEV)
    out = b.run(x)
    for l in range(len(ds)):
        single, stg = q.pipeline(torch.tensor(xs[l], dtype=dt, device=DEV), Bs[l], eps, R)
        assert rel(b.line(out, l).cpu().numpy(), single.cpu().numpy()) <= 1e-11, l
        assert b.ranks(l, 2) == stg["z"].ranks_host()


def test_batch_workload_sample_lines(q):
    """The batched workload itself (4096 lines of 2^10..2^16 samples, 8-32
    scatterers, per-line bandwidths U(100, 2000), FP32, eps 1e-4, R = 32) in one
    batch; every 128th line against the oracle: signal and rounding ranks exact
    wherever the oracle's decision is not a near-tie (relative margin > 1e-5),
    output within the FP32 bound."""
    n = 4096
    ds, Bs, xs, _ = G.batch_lines(n)
    print("workload batch", n, sum(1 << v for v in ds), flush=True)
    dt = torch.float32
    b = q.Batch(ds, Bs, dt, 1e-4, 32, device=DEV)
    x = torch.tensor(np.concatenate(xs), dtype=dt, device=DEV)
    out = b.run(x)
    torch.cuda.synchronize()
    assert int(b.status().abs().sum()) == 0
    for l in range(5, n, 128):
        ref = P.pipeline_1d(xs[l], Bs[l], 1e-4, 32)
        if ref["F_info"]["margin"] > 1e-5:
            assert b.ranks(l, 0) == ref["F_ranks"], (l, ds[l])
        if ref["Z_info"]["margin"] > 1e-5:
            assert b.ranks(l, 2) == ref["Z_ranks"], (l, ds[l])
        got = b.line(out, l).double().cpu().numpy()
        assert rel(got, ref["out"]) <= 2e-4, (l, ds[l], rel(got, ref["out"]))


def test_batch_rejects_bad_plans(q):
    with pytest.raises(q.QttError):
        q.Batch([4, 0], [1.0, 2.0], torch.float32)
    with pytest.raises(q.QttError):
        q.Batch([4, 5], [1.0, -2.0], torch.float32)
    with pytest.raises(q.QttError):
        q.Batch([4, 19], [1.0, 2.0], torch.float32)
    b = q.Batch([4, 5], [1.0, 2.0], torch.float32, device=DEV)
    with pytest.raises(q.QttError):
        b.run(torch.zeros(10, dtype=torch.float32, device=DEV))
