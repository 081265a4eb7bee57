"""Pins of the randomized forms (Algorithms 4 and 5, Appendix A) and of the
counter-based generator that defines their Gaussian test matrices."""

import numpy as np
import pytest

from oracle import rsvd, tt


# Known-answer vectors of Philox-4x32-10 published with the generator
# (Salmon et al. 2011, Random123 test vectors): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = rsvd.philox4x32_10(list(ctr), list(key))
    assert [int(v) for v in got] == list(want)


def test_gaussian_matrix_moments_and_determinism():
    om = rsvd.gaussian_matrix(2000, 50, step=3, seed=12345)
    assert abs(om.mean()) < 0.02 and abs(om.var() - 1.0) < 0.03
    assert np.array_equal(om, rsvd.gaussian_matrix(2000, 50, step=3, seed=12345))
    assert not np.array_equal(om, rsvd.gaussian_matrix(2000, 50, step=4, seed=12345))
    # one entry recomputed from its own counter
    x = rsvd.philox4x32_10([17, 9, 3, 0], [12345, 0])
    u1 = (float(x[0]) + 0.5) * 2.0 ** -32
    u2 = (float(x[1]) + 0.5) * 2.0 ** -32
    assert om[17, 9] == pytest.approx(np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2), rel=1e-15)


def test_rsvd_exact_when_sketch_covers_the_rank():
    """rank(A) <= ell: Q spans range(A) and Algorithm 5 returns the SVD."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 6)) @ rng.standard_normal((6, 300))
    Q = rsvd.range_finder(A, rsvd.gaussian_matrix(300, 10, 1, 7))
    U, s, Vt = rsvd.rsvd(A, Q)
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s[:6], s_ref[:6], rtol=1e-12)
    assert np.allclose((U * s) @ Vt, A, atol=1e-10 * np.linalg.norm(A))


def test_rsvd_error_bound_a1():
    """(A.1): ||A - Q Q^T A|| <= (1 + 11 sqrt(k+p) sqrt(min(m,n))) sigma_{k+1}."""
    rng = np.random.default_rng(1)
    m, n, k, p = 60, 400, 8, 6
    Uo, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, m)))
    sig = np.concatenate([np.geomspace(10.0, 1.0, k), 1e-3 * np.ones(m - k)])
    A = (Uo * sig) @ Vo.T
    for seed in range(5):
        Q = rsvd.range_finder(A, rsvd.gaussian_matrix(n, k + p, 1, seed))
        err = np.linalg.norm(A - Q @ (Q.T @ A), 2)
        assert err <= (1 + 11 * np.sqrt(k + p) * np.sqrt(min(m, n))) * sig[k]


def test_sketched_ttsvd_equals_ttsvd_when_ell_covers_unfoldings():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(1 << 10)
    a, ia = tt.tt_svd(x, 1e-2, 0, return_info=True)
    b, ib = rsvd.tt_svd_sketch(x, 1e-2, 0, ell=64, seed=3, return_info=True)
    assert ia["ranks"] == ib["ranks"]
    assert np.allclose(tt.tt_full(a), tt.tt_full(b), atol=1e-12 * np.linalg.norm(x))


def test_sketched_ttsvd_near_optimal_on_smooth_data():
    """With ell below some unfoldings' row count the sweep is approximate but
    stays within the tolerance on a fast-decaying spectrum."""
    n = 1 << 12
    t = np.arange(n) / n
    x = np.exp(-((t - 0.3) ** 2) / 0.01) + 0.5 * np.sin(40 * t) * t
    eps = 1e-6
    b = rsvd.tt_svd_sketch(x, eps, 0, ell=12, seed=5)
    err = np.linalg.norm(tt.tt_full(b) - x) / np.linalg.norm(x)
    assert err <= 2 * eps


@pytest.mark.parametrize("block", [1, 7, 64, 1 << 15])
def test_sketch_product_blocks_equal_the_whole_test_matrix(block):
    """Y = A Omega summed over row blocks of Omega equals the product with the
    whole matrix of gaussian_matrix (the same entries, another summation order)."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((9, 300))
    want = A @ rsvd.gaussian_matrix(300, 11, 4, 99)
    got = rsvd.sketch_product(A, 11, 4, 99, block=block)
    assert np.allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_range_finder_with_ell_at_least_m_is_the_exact_svd():
    """Algorithm 4 with ell >= m: Y spans R^m, so Algorithm 5 returns the exact
    singular values and the same leading subspaces as the SVD of A (the
    reading that lets the sketched sweep take the exact step there)."""
    rng = np.random.default_rng(4)
    m, n = 12, 500
    A = (rng.standard_normal((m, m)) * np.geomspace(1, 1e-3, m)) @ rng.standard_normal((m, n))
    for ell in (m, m + 4, 64):
        Q = rsvd.range_finder(A, rsvd.gaussian_matrix(n, ell, 2, 5))
        U, s, Vt = rsvd.rsvd(A, Q)
        U0, s0, Vt0 = np.linalg.svd(A, full_matrices=False)
        assert np.allclose(s[:m], s0, rtol=1e-12, atol=0)
        for r in (1, 4, 9):
            P, P0 = U[:, :r] @ U[:, :r].T, U0[:, :r] @ U0[:, :r].T
            assert np.abs(P - P0).max() <= 1e-10


def _sweep_always_sketching(x, eps, ell, seed):
    """The sketched sweep with Algorithms 4/5 at every step, Omega drawn whole."""
    v = np.asarray(x, dtype=np.float64)
    K = tt.log2_exact(v.size)
    tau = eps * np.linalg.norm(v) / np.sqrt(K - 1)
    cores, ranks, r_prev = [], [1], 1
    rem = v.reshape((1, -1), order="F")
    for k in range(1, K):
        A = rem.reshape((2 * r_prev, -1), order="F")
        Q = rsvd.range_finder(A, rsvd.gaussian_matrix(A.shape[1], ell, k, seed))
        U, s, Vt = rsvd.rsvd(A, Q)
        r = tt.truncation_rank(s, tau, 0)
        cores.append(U[:, :r].reshape((r_prev, 2, r), order="F"))
        rem = s[:r, None] * Vt[:r, :]
        ranks.append(r)
        r_prev = r
    cores.append(rem.reshape((r_prev, 2, 1), order="F"))
    return cores, ranks + [1]


def test_sketched_sweep_matches_the_literal_algorithms():
    """tt_svd_sketch (exact step where ell >= m, blocked sketch product
    elsewhere) against the sweep that applies Algorithms 4/5 at every step
    with the whole test matrix: same ranks and tensor."""
    n = 1 << 12
    t = np.arange(n) / n
    rng = np.random.default_rng(6)
    x = np.exp(-((t - 0.3) ** 2) / 0.002) + 0.4 * np.cos(50 * t) + 1e-3 * rng.standard_normal(n)
    eps, ell, seed = 1e-3, 10, 8
    b, info = rsvd.tt_svd_sketch(x, eps, 0, ell=ell, seed=seed, return_info=True)
    c, ranks = _sweep_always_sketching(x, eps, ell, seed)
    assert info["sketched"], "the case must reach steps with ell < m"
    assert info["margin"] > 1e-6
    assert info["ranks"] == ranks
    assert np.linalg.norm(tt.tt_full(b) - tt.tt_full(c)) <= 1e-10 * np.linalg.norm(x)


def test_round_bf16_known_values():
    """bfloat16 keeps 8 significant bits: neighbours of 1 are 1 - 2^-8 and 1 + 2^-7;
    halfway cases go to the even significand."""
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -8, 1.0),                           # halfway, 1 is even
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),           # halfway, round up to even
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above halfway
        (-3.0, -3.0),
        (0.1, 0.10009765625),                             # 0x3DCD in bfloat16
        (0.0, 0.0),
        (2.0 ** -130, 2.0 ** -130),                        # subnormal in float32, exact
    ]
    for x, want in cases:
        assert rsvd.round_bf16(np.array([x]))[0] == want, x
    rng = np.random.default_rng(5)
    v = rng.standard_normal(10000) * 10.0 ** rng.uniform(-20, 20, 10000)
    r = rsvd.round_bf16(v)
    assert np.all(np.abs(r - v) <= 2.0 ** -8 * np.abs(v))
    assert np.array_equal(rsvd.round_bf16(r), r)


def test_sketch_product_bf16_operands_is_the_product_of_rounded_values():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((6, 200))
    om = rsvd.gaussian_matrix(200, 5, 3, 17)
    want = rsvd.round_bf16(A) @ rsvd.round_bf16(om)
    got = rsvd.sketch_product(A, 5, 3, 17, block=64, operands="bf16")
    assert np.allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())
    # the rounding moves the sketch by about 2^-8 relative, not more
    full = A @ om
    assert np.linalg.norm(got - full) <= 2.0 ** -6 * np.linalg.norm(full)


def test_sketched_sweep_with_rounded_operands_is_near_optimal():
    """A sum of five rank-1 QTT terms (ranks <= 5) sketched with ell = 8 below the
    row counts: with operands rounded to single precision or bfloat16 the kept
    subspaces tilt by about that format's unit roundoff, so the tensor is
    recovered to about 1e-6 or 1e-2; exact operands recover it to rounding."""
    d = 12
    rng = np.random.default_rng(9)
    x = np.zeros(1 << d)
    for _ in range(5):
        t = np.ones(1)
        for _k in range(d):
            t = np.concatenate([t * rng.uniform(0.5, 1.5), t * rng.uniform(-1.5, 1.5)])
        x += t
    err = {}
    for ops in ("f64", "f32", "bf16"):
        cores, info = rsvd.tt_svd_sketch(x, 0.0, 5, ell=8, seed=4, return_info=True,
                                         operands=ops)
        assert info["sketched"] and max(info["ranks"]) == 5
        err[ops] = np.linalg.norm(tt.tt_full(cores) - x) / np.linalg.norm(x)
    assert err["f64"] <= 1e-12
    assert err["f32"] <= 1e-5
    assert err["bf16"] <= 3e-2
    assert err["f64"] < err["f32"] < err["bf16"]
