"""GPU parity of the randomised rounding (precision form): the sketched
TT-SVD sweep against the FP64 oracle of Algorithms 4 and 5 with the same
Philox Gaussian matrices."""

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


# a rank decision of the sketch is declared a tie when the oracle's tail sum
# lies within this relative distance of the threshold: with the operands
# rounded alike on both sides, the GPU's FP32 accumulation of the sketch
# perturbs sigma(B)^2 by about 1e-6 relative
TIE = 1e-4


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("method", ["sketch_f32", "sketch_bf16"])
def test_sketch_equals_exact_when_ell_covers(q, method, dt):
    """ell >= every unfolding's row count: each step is the exact SVD, so the
    result is the exact pipeline's (FP64 Gram and eigensolver)."""
    d, B, eps = 12, 200.0, 1e-3
    noisy, _ = G.gaussian_bumps_1d(d, seed=1)
    ref = P.pipeline_1d(noisy, B, eps, 32)
    x = torch.tensor(noisy, dtype=dt, device=DEV)
    out, st = q.pipeline(x, B, eps, 32, round_method=method, sketch_ell=64, sketch_seed=7)
    tol = 1e-10 if dt == torch.float64 else 1e-5
    assert st["z"].ranks_host() == ref["Z_ranks"]
    assert rel(out.cpu().numpy(), ref["out"]) <= tol


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("method,ell", [("sketch_f32", 12), ("sketch_f32", 24),
                                        ("sketch_bf16", 12), ("sketch_bf16", 24)])
def test_sketch_matches_oracle_sketch(q, method, ell, dt):
    """ell below some unfoldings' row count: the same Omega on both sides.  The
    rank decisions are compared with the oracle sketch whose product operands
    are rounded as the GPU's are (single precision or bfloat16), so both sides
    take them on the same values; the output is compared with the FP64-operand
    oracle sketch within the method's tolerance."""
    d, B, eps, seed = 14, 400.0, 1e-4, 11
    noisy, _ = G.scatterers_1d(d, seed=3)
    ref = P.pipeline_1d(noisy, B, eps, 32, sketch_ell=ell, sketch_seed=seed)
    same = P.pipeline_1d(noisy, B, eps, 32, sketch_ell=ell, sketch_seed=seed,
                         sketch_operands="f32" if method == "sketch_f32" else "bf16")
    x = torch.tensor(noisy, dtype=dt, device=DEV)
    out, st = q.pipeline(x, B, eps, 32, round_method=method, sketch_ell=ell, sketch_seed=seed)
    got = out.cpu().numpy()
    err = rel(got, ref["out"])
    tol = max(2 * eps, 1e-5) if method == "sketch_f32" else max(2 * eps, 3e-3)
    gr = st["z"].ranks_host()
    margin = same["Z_info"]["margin"]
    print(f"{method} ell={ell} {dt}: rel {err:.3e} ranks {gr} vs {same['Z_ranks']} "
          f"(decision margin {margin:.2e})", flush=True)
    if margin >= TIE:
        assert gr == same["Z_ranks"]
    else:  # a declared tie: the sums' rounding may settle it either way
        assert all(abs(a - b) <= 1 for a, b in zip(gr, same["Z_ranks"]))
    if max(ref["Z_ranks"]) < ell:
        assert err <= tol
    else:
        # the sketch width limits the rank: many truncations are (almost)
        # equally good, so check near-optimality against the exact rounding
        # instead of agreement with one of them
        exact = P.pipeline_1d(noisy, B, eps, 32)["out"]
        e_gpu, e_ref = rel(got, exact), rel(ref["out"], exact)
        print(f"   sketch-limited: error to the exact rounding {e_gpu:.3e} (oracle sketch "
              f"{e_ref:.3e})", flush=True)
        assert e_gpu <= 1.2 * e_ref + 1e-6


def test_sketch_round_of_exact_tensor_is_accurate(q):
    """Rounding a low-rank tensor given with redundant ranks: the sketched
    sweep recovers it within the tolerance."""
    from oracle import tt
    d = 12
    n = 1 << d
    t = np.arange(n) / n
    v = np.exp(-((t - 0.4) ** 2) / 0.02) + 0.3 * np.cos(9 * t)
    cores = tt.tt_svd(v, 1e-12)
    doubled = tt.tt_from_cores_sum(cores, cores)
    y = q.from_cores(doubled, torch.float64, DEV)
    z = q.round(y, 1e-8, 0, "sketch_bf16", seed=3, ell=16)
    got = q.full(z).cpu().numpy()
    assert rel(got, 2 * v) <= 1e-6


def test_sketch_image_bf16(q):
    """A 256 x 256 image (row-major, separable sinc kernel): BF16 sketch
    rounding against the oracle sketch, and the error to the clean image's
    convolution is the oracle's."""
    dy = dx = 8
    noisy, clean = G.sar_image_2d(dy, dx, seed=3, n_scatterers=20)
    eps, R, ell, seed = 1e-3, 32, 24, 5
    ref = P.pipeline_2d(noisy, 60.0, 60.0, eps, R, sketch_ell=ell, sketch_seed=seed)
    x = torch.tensor(noisy, dtype=torch.float32, device=DEV)
    out, st = q.pipeline(x.reshape(-1), (60.0, 60.0), eps, R, shape2d=noisy.shape,
                         round_method="sketch_bf16", sketch_ell=ell, sketch_seed=seed)
    assert rel(out.cpu().numpy(), ref["out"]) <= max(2 * eps, 3e-3)


@pytest.fixture(scope="module")
def image4096():
    noisy, clean = G.sar_image_2d(12, 12, seed=3)
    return noisy, clean


def test_image_4096_exact_forms_against_the_oracle(q, image4096):
    """The 4096 x 4096 image at full size (24 binary modes, separable sinc
    Bx = By = 1000, eps = 1e-3, R = 32) through the exact pipeline: FP64 within
    1e-10 of the oracle's FP64 pipeline with the same ranks; FP32 data within
    max(2 eps, 1e-5); the BF16-operand sketch rounding (ell = 64) within
    max(2 eps, 3e-3) of the same oracle."""
    noisy, _ = image4096
    eps, R, B = 1e-3, 32, 1000.0
    print("case: image 4096 exact forms", flush=True)
    ref = P.pipeline_2d(noisy, B, B, eps, R)
    x64 = torch.tensor(noisy, dtype=torch.float64, device=DEV)
    out, st = q.pipeline(x64, (B, B), eps, R, shape2d=noisy.shape)
    e64 = rel(out.cpu().numpy(), ref["out"])
    print(f"FP64: rel {e64:.3e} Z ranks {st['z'].ranks_host()} oracle {ref['Z_ranks']} margins "
          f"{ref['F_info']['margin']:.2e} {ref['Z_info']['margin']:.2e}", flush=True)
    assert st["f"].ranks_host() == ref["F_ranks"]
    assert st["z"].ranks_host() == ref["Z_ranks"]
    assert e64 <= 1e-10
    del out, x64
    x32 = torch.tensor(noisy, dtype=torch.float32, device=DEV)
    o32, st32 = q.pipeline(x32, (B, B), eps, R, shape2d=noisy.shape)
    e32 = rel(o32.cpu().numpy(), ref["out"])
    ob, stb = q.pipeline(x32, (B, B), eps, R, shape2d=noisy.shape, round_method="sketch_bf16",
                         sketch_ell=64, sketch_seed=1)
    eb = rel(ob.cpu().numpy(), ref["out"])
    print(f"FP32 exact: rel {e32:.3e}; BF16 sketch: rel {eb:.3e} ranks {stb['z'].ranks_host()}",
          flush=True)
    assert e32 <= max(2 * eps, 1e-5)
    assert eb <= max(2 * eps, 3e-3)
    for s_ in (st32, stb):
        assert s_["z"].status_host() == 0 and s_["f"].status_host() == 0




def test_image_4096_sketch_against_the_oracle_sketch(q, image4096):
    """The BF16 and FP32 sketch roundings of the full-size image against the
    oracle's sketch sweep with the same Omega (Philox, seed 1, ell = 64; the
    oracle takes the exact step where ell covers the rows): ranks exact unless
    a decision is a declared tie, outputs within the method's tolerance."""
    noisy, _ = image4096
    eps, R, B, ell = 1e-3, 32, 1000.0, 64
    print("case: image 4096 sketch vs oracle sketch", flush=True)
    x32 = torch.tensor(noisy, dtype=torch.float32, device=DEV)
    noisy32 = noisy.astype(np.float32).astype(np.float64)
    for method, ops in (("sketch_f32", "f32"), ("sketch_bf16", "bf16")):
        ref = P.pipeline_2d(noisy32, B, B, eps, R, sketch_ell=ell, sketch_seed=1,
                            sketch_operands=ops)
        margin = ref["Z_info"]["margin"]
        out, st = q.pipeline(x32, (B, B), eps, R, shape2d=noisy.shape, round_method=method,
                             sketch_ell=ell, sketch_seed=1)
        err = rel(out.cpu().numpy(), ref["out"])
        gr = st["z"].ranks_host()
        print(f"{method}: rel {err:.3e} ranks {gr} oracle {ref['Z_ranks']} margin {margin:.2e} "
              f"sketched steps {ref['Z_info']['sketched']}", flush=True)
        assert ref["Z_info"]["sketched"], "the case must reach sketched steps"
        if margin >= TIE:
            assert gr == ref["Z_ranks"]
        else:
            assert all(abs(a - b) <= 1 for a, b in zip(gr, ref["Z_ranks"]))
        assert err <= (max(2 * eps, 1e-5) if method == "sketch_f32" else max(2 * eps, 3e-3))
