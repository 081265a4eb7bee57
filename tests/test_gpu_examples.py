"""The paper's Examples 1 and 2 (Section 7) end to end on the GPU.

Each example runs the GPU pipeline with the max-rank truncation (R_max = 10,
rounding capped at 15 as the paper caps its QTT-FFT) and with the
singular-value drop-off of modification (3) (the paper's thresholds), on the
paper's grid (N = 2^(K-1) - 1 noisy samples zero-padded to 2^K, K = 20, kernel
resolution 4 dx and 2 dx).  The output is compared with the FP64 oracle
pipeline on the same input (ranks exact, FP64 to 1e-10; 1e-6 for the drop-off
runs, where the rank cap binds on noise-level spectra), and its error (7.1)
against the noise-free convolution is checked to show the denoising the
paper reports: far below the error of convolving the noisy data, and within
a factor of two of Table 7.1 (context only: the paper convolves by QTT-FFT).
"""

import json
import os

import numpy as np
import pytest

from oracle import pipeline as P
from synthetic import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_13339_amd as q  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "table_7_1_qtt_errors.json")))["values"]
K = 20
GENS = {"example1": G.paper_example1, "example2": G.paper_example2}


def _inputs(name):
    noisy, clean, _, _ = GENS[name](K, 0)
    x = np.zeros(1 << K)
    c = np.zeros(1 << K)
    x[: noisy.size] = noisy
    c[: clean.size] = clean
    B = (1 << K) / float(GOLD[name]["resolution_in_dx"])
    return x, c, B


@pytest.mark.parametrize("name", ["example1", "example2"])
@pytest.mark.parametrize("rule", ["max_rank", "dropoff"])
def test_paper_example(name, rule):
    print("case: example", name, rule, flush=True)
    x, c, B = _inputs(name)
    if rule == "max_rank":
        kw = dict(eps=1e-4, max_rank=10, round_max_rank=15, delta=0.0)
    else:
        kw = dict(eps=0.0, max_rank=64, round_max_rank=64, delta=GOLD[name]["delta_threshold"])
    ref = P.pipeline_1d(x, B, kw["eps"], max_rank=kw["max_rank"],
                        round_max_rank=kw["round_max_rank"], delta=kw["delta"])
    out, st = q.pipeline(torch.tensor(x, device="cuda"), B, kw["eps"], kw["max_rank"],
                         round_max_rank=kw["round_max_rank"], delta=kw["delta"])
    out = out.cpu().numpy()
    assert st["f"].ranks_host() == ref["F_ranks"]
    assert st["z"].ranks_host() == ref["Z_ranks"]
    # with the drop-off alone nothing truncates the noise floor of the fine
    # unfoldings, so the cap of 64 binds there on clustered noise-level
    # singular values; the kept subspace is then fixed by the Gram route
    # only to about u sigma_1^2 / (sigma_64^2 - sigma_65^2) (measured 1e-8)
    tol = 1e-10 if rule == "max_rank" else 1e-6
    assert P.relative_error(out, ref["out"]) <= tol
    clean_conv = P.clean_reference_1d(c, B)
    e_noisy = P.relative_error(P.clean_reference_1d(x, B), clean_conv)
    e = P.relative_error(out, clean_conv)
    table = GOLD[name]["qtt0" if rule == "max_rank" else "delta"]
    print(f"E2 {name} {rule}: {e:.4f} (noisy convolution {e_noisy:.4f}, Table 7.1 {table})",
          flush=True)
    assert e < 0.6 * e_noisy
    assert 0.5 * table <= e <= 2.0 * table
