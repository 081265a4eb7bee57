"""Pins of the general-mode TT-SVD and max-rank TT-RSVD (Section 5, modifications
(1) and (2); Algorithms 1, 4, 5): the binary special case equals the QTT oracle,
eps = 0 is exact, the truncation error identity, closed-form ranks of sums of
outer products, entry products against Full, and the randomised sweep exact on
tensors whose ranks the sketch covers."""

import numpy as np
import pytest

from oracle import rsvd, tt, ttm


def _outer(vecs):
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out  # C order, last mode slowest in flattening order F


def _tensor_from_terms(modes, nterms, seed):
    rng = np.random.default_rng(seed)
    a = np.zeros(modes)
    for _ in range(nterms):
        a += _outer([rng.standard_normal(m) for m in modes])
    return a


def test_binary_modes_equal_qtt_oracle():
    x = np.random.default_rng(0).standard_normal(1 << 10)
    for eps, cap in ((1e-2, 0), (0.0, 5), (1e-6, 0)):
        a, ia = ttm.tt_svd_modes(x, [2] * 10, eps, cap, return_info=True)
        b, ib = tt.tt_svd(x, eps, cap, return_info=True)
        assert ia["ranks"] == ib["ranks"]
        for ca, cb in zip(a, b):
            assert np.allclose(ca, cb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("modes", [(3, 4, 5), (10, 10, 10, 10), (7, 2, 9, 3, 5)])
def test_eps0_exact_and_entries(modes):
    a = np.random.default_rng(1).standard_normal(modes)
    cores = ttm.tt_svd_modes(a, modes, 0.0)
    full = ttm.tt_full_modes(cores)
    flat = a.ravel(order="F")
    assert np.max(np.abs(full - flat)) <= 1e-12 * np.max(np.abs(flat))
    idx = np.random.default_rng(2).integers(0, flat.size, 20)
    for i in idx:
        assert ttm.tt_entry_modes(cores, int(i)) == pytest.approx(full[i], rel=1e-12, abs=1e-12)


def test_error_identity():
    """||a - a_TT||^2 equals the sum of the discarded squared singular values (exact SVD)."""
    modes = (6, 6, 6, 6)
    a = np.random.default_rng(3).standard_normal(modes)
    cores, info = ttm.tt_svd_modes(a, modes, 0.3, return_info=True)
    disc = sum(float(np.sum(s[r:] ** 2)) for s, r in zip(info["sv"], info["ranks"][1:]))
    err = float(np.sum((ttm.tt_full_modes(cores) - a.ravel(order="F")) ** 2))
    assert err == pytest.approx(disc, rel=1e-9)
    assert np.sqrt(err) <= 0.3 * info["norm"] * (1 + 1e-12)


@pytest.mark.parametrize("nterms", [1, 2, 3])
def test_sum_of_outer_products_ranks(nterms):
    modes = (5, 8, 6, 7)
    a = _tensor_from_terms(modes, nterms, 4)
    cores, info = ttm.tt_svd_modes(a, modes, 1e-10, return_info=True)
    want = [1] + [min(nterms, int(np.prod(modes[:k])), int(np.prod(modes[k:])))
                  for k in range(1, len(modes))] + [1]
    assert info["ranks"] == want


def test_rsvd_exact_on_low_rank_tensor():
    """Ranks <= R: the sketch (ell = R + p) spans each unfolding's range, so the
    randomised sweep reproduces the tensor and the exact sweep's singular values."""
    modes = (10, 10, 10, 10, 10)
    a = _tensor_from_terms(modes, 4, 5)
    R, p = 6, 4
    c_r, i_r = ttm.tt_svd_modes(a, modes, 0.0, R, True, method="rsvd", oversample=p, seed=9)
    c_s, i_s = ttm.tt_svd_modes(a, modes, 0.0, R, True)
    assert not all(i_r["exact_steps"])           # some steps are randomised
    flat = a.ravel(order="F")
    assert np.linalg.norm(ttm.tt_full_modes(c_r) - flat) <= 1e-11 * np.linalg.norm(flat)
    for s_r, s_s, r in zip(i_r["sv"], i_s["sv"], i_r["ranks"][1:]):
        assert np.allclose(s_r[:r], s_s[:r], rtol=1e-10, atol=1e-12 * s_s[0])


def test_rsvd_reverts_to_svd_on_small_unfoldings():
    """min(m_k, n_k) <= R + p: every step is the exact SVD, as Section 5 prescribes."""
    modes = (4, 5, 4)
    a = np.random.default_rng(6).standard_normal(modes)
    c_r, i_r = ttm.tt_svd_modes(a, modes, 1e-3, 8, True, method="rsvd", oversample=4)
    c_s, i_s = ttm.tt_svd_modes(a, modes, 1e-3, 8, True)
    assert all(i_r["exact_steps"])
    assert i_r["ranks"] == i_s["ranks"]
    for x, y in zip(c_r, c_s):
        assert np.array_equal(x, y)


def test_rsvd_step_within_the_expected_bound():
    """One randomised step on a decaying spectrum: ||A - Q Q^T A||_F within a small factor of
    (1 + k / (p - 1))^(1/2) (sum_{j > k} sigma_j^2)^(1/2) (the expected bound of HMT Thm 10.5)."""
    rng = np.random.default_rng(7)
    m, n, k, p = 60, 400, 8, 6
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, m)))
    s = 0.7 ** np.arange(m)
    A = (U * s) @ V.T
    Q = rsvd.range_finder(A, rsvd.gaussian_matrix(n, k + p, 1, 11))
    err = np.linalg.norm(A - Q @ (Q.T @ A))
    bound = np.sqrt(1 + k / (p - 1)) * np.sqrt(np.sum(s[k:] ** 2))
    assert err <= 3 * bound
    assert err >= np.sqrt(np.sum(s[k + p:] ** 2)) * (1 - 1e-9)   # no projector beats the SVD
