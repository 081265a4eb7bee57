"""Pins of the oracle's TT algorithms (Algorithm 1, Algorithm 3, TT-rounding).

Each test checks the oracle against something other than itself: closed-form
ranks, the exact error identity of truncated SVDs, brute-force entry
products, the paper's printed ranks and storage counts.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import tt
from synthetic import generators as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _rand_cores(ranks, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((ranks[k], 2, ranks[k + 1])) for k in range(len(ranks) - 1)]


# ---------------------------------------------------------------- rank rule

def test_truncation_rank_rule():
    s = np.array([4.0, 3.0, 2.0, 1.0])
    # tails: r=1 -> 9+4+1=14, r=2 -> 5, r=3 -> 1, r=4 -> 0
    assert tt.truncation_rank(s, 0.0) == 4
    assert tt.truncation_rank(s, 1.0) == 3          # equality keeps the smaller rank
    assert tt.truncation_rank(s, math.sqrt(5.0)) == 2
    assert tt.truncation_rank(s, 0.999) == 4
    assert tt.truncation_rank(s, 100.0) == 1         # never below 1
    assert tt.truncation_rank(s, 0.0, max_rank=2) == 2
    assert tt.truncation_rank(np.zeros(3), 0.0) == 1


# ---------------------------------------------------------------- Algorithm 3

@pytest.mark.parametrize("d", [1, 2, 5, 10])
def test_full_matches_entry_products(d):
    rng = np.random.default_rng(d)
    ranks = [1] + [int(rng.integers(1, 5)) for _ in range(d - 1)] + [1]
    cores = _rand_cores(ranks, d)
    v = tt.tt_full(cores)
    assert v.size == 1 << d
    idx = range(v.size) if d <= 5 else rng.integers(0, v.size, 200)
    for i in idx:
        assert abs(v[i] - tt.tt_entry(cores, int(i))) <= 1e-12 * (1 + abs(v[i]))


def test_full_bit_order_lsb_first():
    # rank-1 tensor whose mode k carries factor (1, 2**(2**(k-1)))-like weights:
    # v(i) = prod_k a_k[i_k] with a_k = (1, 10**k)  =>  v(i) = 10**(sum_k k i_k)
    d = 4
    cores = [np.array([1.0, 10.0 ** (k + 1)]).reshape(1, 2, 1) for k in range(d)]
    v = tt.tt_full(cores)
    for i in range(1 << d):
        e = sum((k + 1) * ((i >> k) & 1) for k in range(d))
        assert v[i] == pytest.approx(10.0 ** e)


# ---------------------------------------------------------------- Algorithm 1

@pytest.mark.parametrize("d", [1, 2, 3, 7, 10])
def test_ttsvd_eps0_exact(d):
    x = np.random.default_rng(10 + d).standard_normal(1 << d)
    cores = tt.tt_svd(x, 0.0)
    assert np.max(np.abs(tt.tt_full(cores) - x)) <= 1e-13 * np.max(np.abs(x)) * 10


@pytest.mark.parametrize("eps,cap", [(1e-1, 0), (3e-2, 0), (1e-2, 6), (0.0, 3), (0.2, 2)])
def test_ttsvd_error_identity(eps, cap):
    """||A - A_TT||_F^2 equals the sum of all discarded squared singular values."""
    d = 10
    x = G.gaussian_bumps_1d(d, seed=7)[0]
    cores, info = tt.tt_svd(x, eps, cap, return_info=True)
    err2 = np.sum((tt.tt_full(cores) - x) ** 2)
    disc = sum(np.sum(s[r:] ** 2) for s, r in zip(info["sv"], info["ranks"][1:-1]))
    assert err2 == pytest.approx(disc, rel=1e-9, abs=1e-24 * np.sum(x * x))
    if cap == 0:
        assert math.sqrt(err2) <= eps * np.linalg.norm(x) * (1 + 1e-12)


def test_ttsvd_unfolding_shapes_lemma_5_1():
    d, R = 12, 5
    x = np.random.default_rng(3).standard_normal(1 << d)
    cores, info = tt.tt_svd(x, 1e-6, R, return_info=True)
    r = info["ranks"]
    for k in range(1, d):
        m_k, n_k = 2 * r[k - 1], 1 << (d - k)
        assert m_k <= 2 * R
        assert len(info["sv"][k - 1]) == min(m_k, n_k)
    assert [c.shape for c in cores] == [(r[k], 2, r[k + 1]) for k in range(d)]


@pytest.mark.parametrize("d", [8, 16])
@pytest.mark.parametrize("kind,param,rank", [
    ("exp", 3.0, 1), ("sin", 5.0, 2), ("cos", 2.0, 2),
    ("poly", 1, 2), ("poly", 3, 4), ("poly", 5, 6)])
def test_ttsvd_closed_form_ranks(d, kind, param, rank):
    x = G.closed_form_signal(kind, d, param)
    cores = tt.tt_svd(x, 1e-12)
    assert max(tt.tt_ranks(cores)) == rank
    assert np.linalg.norm(tt.tt_full(cores) - x) <= 1e-11 * np.linalg.norm(x)


def test_ttsvd_zero_tensor():
    cores = tt.tt_svd(np.zeros(64), 1e-3)
    assert tt.tt_ranks(cores) == [1] * 7
    assert np.all(tt.tt_full(cores) == 0)


def test_ttsvd_sign_gauge():
    x = G.gaussian_bumps_1d(8, seed=2)[0]
    cores = tt.tt_svd(x, 1e-2)
    for c in cores[:-1]:
        U = c.reshape((-1, c.shape[2]), order="F")
        for j in range(U.shape[1]):
            assert U[np.argmax(np.abs(U[:, j])), j] > 0


def test_paper_max_ranks_examples():
    gold = _gold("max_qtt_ranks.json")
    eps = gold["eps"]

    def pad(v, n):
        out = np.zeros(n)
        out[: v.size] = v
        return out

    for name, gen in (("example1", G.paper_example1), ("example2", G.paper_example2)):
        _, f, _, _ = gen(20)
        cores = tt.tt_svd(pad(f, 1 << 20), eps)
        assert max(tt.tt_ranks(cores)) == gold["values"][name]
    _, f, _, _ = G.paper_example3(10)
    img = np.zeros((1024, 1024))
    img[: f.shape[0], : f.shape[1]] = f
    # Matlab's column-major reshape of f[j, k] = f(x_j, y_k): the x index varies fastest
    cores = tt.tt_svd(img.ravel(order="F"), eps)
    assert max(tt.tt_ranks(cores)) == gold["values"]["example3"]


def test_threshold_reading_sqrt_K_minus_1():
    """The printed sqrt(M-1) (M = 2) threshold does not reproduce the printed rank 17."""
    _, f, _, _ = G.paper_example1(20)
    v = np.zeros(1 << 20)
    v[: f.size] = f
    _, info = tt.tt_svd(v, 1e-10, return_info=True)
    # with tau = eps*||A|| (sqrt(M-1) = 1) the largest rank would be smaller
    s_all = info["sv"]
    tau1 = 1e-10 * info["norm"]
    r_alt = max(tt.truncation_rank(s, tau1) for s in s_all)
    assert max(info["ranks"]) == 17 and r_alt != 17


def test_storage_counts_tables_7_3_7_5():
    gold = _gold("table_7_3_storage.json")
    R = gold["R_max"]
    for K, count in zip(gold["K"], gold["count"]):
        prof = [1] + [min(1 << k, 1 << (K - k), R) for k in range(1, K)] + [1]
        assert tt.storage_count(prof) == count
    # the max-rank TT-SVD of full-length noisy data produces exactly that profile
    for K, count in zip(gold["K"][:2], gold["count"][:2]):
        noisy, _, _, _ = G.paper_example1(K, seed=1, full_grid=True)
        cores = tt.tt_svd(noisy, 1e-10, R)
        assert tt.storage_count(tt.tt_ranks(cores)) == count


# ---------------------------------------------------------------- rounding

@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6])
def test_round_of_exact_tt_equals_ttsvd(eps):
    d = 11
    x = G.scatterers_1d(d, seed=5, n_scatterers=6)[1]
    exact = tt.tt_svd(x, 0.0)
    # scramble the gauge so the rounding has real work to do
    rng = np.random.default_rng(1)
    g = [c.copy() for c in exact]
    for k in range(d - 1):
        r = g[k].shape[2]
        S = rng.standard_normal((r, r)) + 3 * np.eye(r)
        g[k] = np.einsum("aib,bc->aic", g[k], S)
        g[k + 1] = np.einsum("ab,bic->aic", np.linalg.inv(S), g[k + 1])
    Zr, rinfo = tt.tt_round(g, eps, return_info=True)
    Zs, sinfo = tt.tt_svd(x, eps, return_info=True)
    assert rinfo["ranks"] == sinfo["ranks"]
    assert np.linalg.norm(tt.tt_full(Zr) - tt.tt_full(Zs)) <= 1e-11 * np.linalg.norm(x)


def test_round_redundant_sum():
    d = 10
    x = G.closed_form_signal("sin", d, 3.0) + 0.5 * G.closed_form_signal("exp", d, 1.0)
    X = tt.tt_svd(x, 1e-13)
    S = tt.tt_from_cores_sum(X, X)
    assert max(tt.tt_ranks(S)) == 2 * max(tt.tt_ranks(X))
    Z = tt.tt_round(S, 1e-12)
    assert tt.tt_ranks(Z) == tt.tt_ranks(X)
    assert np.linalg.norm(tt.tt_full(Z) - 2 * x) <= 1e-11 * np.linalg.norm(x)


def test_round_cores_left_orthonormal():
    cores = _rand_cores([1, 2, 4, 6, 5, 3, 2, 1], 4)
    Z = tt.tt_round(cores, 1e-3)
    for c in Z[:-1]:
        U = c.reshape(-1, c.shape[2])
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= 1e-13
    assert np.linalg.norm(Z[-1]) == pytest.approx(np.linalg.norm(tt.tt_full(Z)), rel=1e-12)


# ------------------------------------------- drop-off rule, modification (3)

def test_dropoff_rank_definition():
    """The first ratio s_{k+1}/s_k below delta keeps k values (Section 5, modification (3))."""
    s = np.array([1.0, 0.5, 0.2, 0.01, 0.009])
    # ratios 0.5, 0.4, 0.05, 0.9
    assert tt.dropoff_rank(s, 0.3) == 3
    assert tt.dropoff_rank(s, 0.45) == 2      # 0.4 < 0.45 comes before 0.05
    assert tt.dropoff_rank(s, 0.55) == 1
    assert tt.dropoff_rank(s, 0.04) is None   # no ratio below 0.04
    assert tt.dropoff_rank(s, 0.0) is None    # off
    # squared ratios would give 1 here (0.25 < 0.3): the rule is on sigma, not sigma^2
    assert tt.dropoff_rank(np.array([1.0, 0.5, 0.6 * 0.5]), 0.3) is None
    # equality is not a drop
    assert tt.dropoff_rank(np.array([1.0, 0.25]), 0.25) is None
    # zero singular values: a drop to zero cuts, 0/0 does not
    assert tt.dropoff_rank(np.array([2.0, 0.0, 0.0]), 0.1) == 1
    assert tt.dropoff_rank(np.array([0.0, 0.0]), 0.1) is None


def _exp_sum(d, rates, amps):
    x = np.arange(1 << d) / float(1 << d)
    return sum(a * np.exp(c * x) for c, a in zip(rates, amps))


@pytest.mark.parametrize("d", [8, 12])
def test_dropoff_recovers_exact_ranks(d):
    """A sum of three exponentials has QTT ranks min(2^k, 2^(d-k), 3); its further
    singular values are rounding noise, so any delta between the noise ratio and the
    smallest genuine ratio recovers exactly those ranks with eps = 0, where the
    tolerance rule alone keeps the rounding noise (full ranks)."""
    v = _exp_sum(d, [-1.0, 2.5, 6.0], [1.0, -0.7, 0.05])
    want = [1] + [min(1 << k, 1 << (d - k), 3) for k in range(1, d)] + [1]
    cores, info = tt.tt_svd(v, 0.0, 0, True, delta=1e-6)
    assert info["ranks"] == want
    rec = tt.tt_full(cores)
    assert np.linalg.norm(rec - v) <= 1e-11 * np.linalg.norm(v)
    # without the cut, eps = 0 keeps the rounding-level singular values
    plain = tt.tt_svd(v, 0.0, 0, True)[1]["ranks"]
    assert max(plain) > 3


def test_dropoff_combines_with_tolerance_and_cap():
    """The kept rank is min(eps-rank, drop-off rank, cap) at every unfolding."""
    _, clean = G.gaussian_bumps_1d(10, seed=7, noise_rel=0.0)
    rng = np.random.default_rng(3)
    x = clean + 1e-3 * rng.standard_normal(clean.size)
    for eps, cap, delta in [(1e-2, 0, 0.3), (1e-4, 0, 0.05), (1e-6, 6, 0.02), (0.0, 0, 0.1)]:
        _, info = tt.tt_svd(x, eps, cap, True, delta=delta)
        tau = info["tau"]
        for k, s in enumerate(info["sv"], start=1):
            r_eps = tt.truncation_rank(s, tau, 0)
            r_d = tt.dropoff_rank(s, delta)
            want = min(r_eps, r_d if r_d is not None else s.size, cap if cap > 0 else s.size)
            assert info["ranks"][k] == max(want, 1)
    # delta = 0 is plain Algorithm 1
    a = tt.tt_svd(x, 1e-3, 0, True)[1]["ranks"]
    b = tt.tt_svd(x, 1e-3, 0, True, delta=0.0)[1]["ranks"]
    assert a == b
