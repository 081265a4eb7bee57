"""Tensor-train algorithms of Section 4 and Section 5, in plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (Section 4, definitions of the TT format, the unfolding and the
QTT reshape):

* A core is a numpy array of shape ``(r_{k-1}, 2, r_k)``; ``core[a, i, b]`` is
  entry ``(a, b)`` of slice ``i``.  ``r_0 = r_K = 1``.
* A vector ``v`` of length ``2**K`` is the ``K``-mode tensor with
  ``v(i) = V(i_1, ..., i_K)``, ``i = sum_k i_k 2**(k-1)`` (``i_1`` is the least
  significant bit).  A row-major image is flattened row-major, so its column
  bits come first.
* ``reshape`` is column-major (Matlab) throughout, as the paper states.

Readings of the text (where it is silent, garbled or inconsistent):

* Algorithm 1 prints the threshold with ``sqrt(M-1)``, ``M`` the largest mode
  size.  For a QTT (``M = 2``) that contradicts the error split
  ``eps^2 = sum_k eps_k^2`` over the ``K-1`` unfoldings stated right before
  it; the threshold used is ``tau = eps * ||A||_F / sqrt(K-1)``.
* "truncated SVD with ``||E||_F <= tau``" is read as: keep the smallest
  ``r >= 1`` whose discarded tail satisfies ``sum_{i>r} sigma_i^2 <= tau^2``
  (equality keeps the smaller rank).  Modification (1) of Section 5 (max
  rank) then takes ``min(r, R_max)``; ``max_rank = 0`` means uncapped.
* Modification (3) of Section 5 (singular-value drop-off) is read as: with
  ``s`` non-increasing, the kept rank is the smallest ``k >= 1`` with
  ``s_{k+1} < delta * s_k`` (1-based; the first relative drop below
  ``delta`` cuts everything after it), and no cut when no ratio is below
  ``delta``.  It is combined with the tolerance rule and the cap as
  ``min(r_eps, r_delta, R_max)``; ``eps = 0`` and no cap give the pure
  drop-off method, ``delta = 0`` turns it off.  A ratio ``0 / 0`` (two zero
  singular values) is not a drop.
* Sign gauge (cores are unique only up to it): each kept left singular vector
  is flipped so that its largest-magnitude entry is positive.
* TT-rounding is not described in the paper (only the TT-SVD of O11 is);
  the standard algorithm is used: right-to-left orthogonalisation by LQ,
  then a left-to-right sweep of truncated SVDs with the same rule and the
  threshold computed from the norm of the rounded tensor.
"""

from __future__ import annotations

import math

import numpy as np


def log2_exact(n: int) -> int:
    """``K`` with ``2**K == n``; raises if ``n`` is not a power of two."""
    k = int(n).bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError(f"length {n} is not a power of two")
    return k


def truncation_rank(s: np.ndarray, tau: float, max_rank: int = 0) -> int:
    """Rank kept by a truncated SVD with Frobenius tail ``<= tau``.

    ``s`` holds singular values in non-increasing order.  Returns the
    smallest ``r >= 1`` with ``sum_{i >= r} s_i^2 <= tau^2`` (0-based tail),
    capped at ``max_rank`` when positive (Algorithm 1 and modification (1)).
    """
    s = np.asarray(s, dtype=np.float64)
    n = s.size
    # tail[r] = sum_{i >= r} s_i^2, accumulated from the small end
    tail = np.zeros(n + 1)
    tail[:n] = np.cumsum((s * s)[::-1])[::-1]
    r = n
    for cand in range(1, n + 1):
        if tail[cand] <= tau * tau:
            r = cand
            break
    if max_rank > 0:
        r = min(r, max_rank)
    return max(r, 1)


def dropoff_rank(s: np.ndarray, delta: float):
    """Rank kept by the singular-value drop-off rule, modification (3) of Section 5.

    ``s`` holds singular values in non-increasing order.  Returns the smallest
    ``k >= 1`` with ``s[k] < delta * s[k-1]`` (0-based, i.e. keep ``s[0..k-1]``),
    or ``None`` when no ratio falls below ``delta`` (or ``delta <= 0``).
    """
    if not delta > 0.0:
        return None
    s = np.asarray(s, dtype=np.float64)
    for k in range(1, s.size):
        if s[k] < delta * s[k - 1]:
            return k
    return None


def _gauge(u: np.ndarray, vt: np.ndarray):
    """Flip each column of ``u`` (and row of ``vt``) so its largest |entry| is > 0."""
    for j in range(u.shape[1]):
        i = int(np.argmax(np.abs(u[:, j])))
        if u[i, j] < 0:
            u[:, j] = -u[:, j]
            vt[j, :] = -vt[j, :]
    return u, vt


def tt_svd(a, eps: float, max_rank: int = 0, return_info: bool = False, delta: float = 0.0):
    """Algorithm 1 (TT-SVD) on the QTT reshape of ``a``, with modifications (1) and (3).

    ``a`` is a vector of length ``2**K`` (or a row-major array of that many
    entries).  ``delta > 0`` adds the drop-off cut of modification (3)
    (:func:`dropoff_rank`).  Returns the list of ``K`` cores (and, with
    ``return_info``, a dict with the threshold, ranks, singular values of
    every unfolding, the smallest relative distance ``|tail^2 - tau^2| /
    tau^2`` over the decisions the threshold made, and the smallest
    ``|s[k]/s[k-1] - delta| / delta`` over the ratios the drop-off rule
    examined, both used to flag near-ties).
    """
    v = np.asarray(a, dtype=np.float64).ravel()
    K = log2_exact(v.size)
    norm = float(np.linalg.norm(v))
    info = {"norm": norm, "sv": [], "ranks": [1], "margin": math.inf, "delta_margin": math.inf}
    if K == 1:
        cores = [v.reshape(1, 2, 1).copy()]
        info["tau"] = 0.0
        info["ranks"].append(1)
        return (cores, info) if return_info else cores
    tau = eps * norm / math.sqrt(K - 1)
    info["tau"] = tau
    cores = []
    r_prev = 1
    rem = v.reshape((1, -1), order="F")
    for _k in range(1, K):
        A = rem.reshape((2 * r_prev, -1), order="F")          # unfolding, Lemma 5.1 shape
        U, s, Vt = np.linalg.svd(A, full_matrices=False)
        r = truncation_rank(s, tau, max_rank)
        r_drop = dropoff_rank(s, delta)
        if r_drop is not None:
            r = min(r, r_drop)
        if delta > 0.0:
            # ratios up to the first drop decided the cut (all of them if none)
            last = r_drop if r_drop is not None else s.size - 1
            for j in range(1, last + 1):
                if s[j - 1] > 0.0:
                    info["delta_margin"] = min(info["delta_margin"],
                                               abs(s[j] / s[j - 1] - delta) / delta)
        info["sv"].append(s.copy())
        if tau > 0:
            tails = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
            r_eps = truncation_rank(s, tau, 0)
            if max_rank <= 0 or r_eps <= max_rank:
                # distance of the deciding tails from the threshold
                cand = [tails[r_eps]] + ([tails[r_eps - 1]] if r_eps >= 1 else [])
                for t in cand:
                    info["margin"] = min(info["margin"], abs(t - tau * tau) / (tau * tau))
        U = U[:, :r].copy()
        Vt = Vt[:r, :].copy()
        U, Vt = _gauge(U, Vt)
        cores.append(U.reshape((r_prev, 2, r), order="F"))
        rem = s[:r, None] * Vt                                  # Sigma V^*
        info["ranks"].append(r)
        r_prev = r
    cores.append(rem.reshape((r_prev, 2, 1), order="F"))
    info["ranks"].append(1)
    return (cores, info) if return_info else cores


def tt_full(cores) -> np.ndarray:
    """Algorithm 3 (Full): contract the cores into the vector of length ``2**K``.

    ``A <- reshape(A, [|A|/r_{k-1}, r_{k-1}]) @ reshape(G_k, [r_{k-1}, 2 r_k])``
    for ``k = 2..K`` with column-major reshapes; the result is the vector in
    the QTT index order (least significant bit first).
    """
    A = np.asarray(cores[0], dtype=np.float64)
    A = A.reshape((-1, A.shape[2]), order="F")                # (2, r_1)
    for G in cores[1:]:
        r0, _, r1 = G.shape
        A = A.reshape((-1, r0), order="F")
        B = np.asarray(G, dtype=np.float64).reshape((r0, 2 * r1), order="F")
        A = A @ B
        A = A.reshape((-1, r1), order="F")
    return A.reshape(-1, order="F")


def tt_entry(cores, idx: int) -> float:
    """One entry ``v(idx)`` as the product of core slices (Section 4)."""
    row = np.ones((1, 1))
    for k, G in enumerate(cores):
        row = row @ G[:, (idx >> k) & 1, :]
    return float(row[0, 0])


def tt_ranks(cores):
    """``[r_0, r_1, ..., r_K]``."""
    return [cores[0].shape[0]] + [G.shape[2] for G in cores]


def tt_round(cores, eps: float, max_rank: int = 0, return_info: bool = False):
    """TT-rounding (standard algorithm; the paper cites O11 but gives no text).

    1. Right-to-left, for ``k = K..2``: LQ of ``G_k`` viewed as
       ``r_{k-1} x (2 r_k)``; ``G_k <- Q``; ``G_{k-1} <- G_{k-1} x_3 L``.
    2. ``tau = eps * ||A||_F / sqrt(K-1)`` with the norm of the first core.
    3. Left-to-right, for ``k = 1..K-1``: SVD of ``G_k`` viewed as
       ``(2 r_{k-1}) x r_k``, truncate by :func:`truncation_rank`,
       ``G_k <- U``; ``G_{k+1} <- (Sigma V^*) x_1 G_{k+1}``.

    For an exact TT of ``A`` this returns the same ranks and the same tensor
    as :func:`tt_svd` of ``A`` (the unfoldings seen by both sweeps have the
    same singular values and left singular subspaces).
    """
    G = [np.asarray(c, dtype=np.float64).copy() for c in cores]
    K = len(G)
    info = {"ranks": None, "sv": [], "margin": math.inf}
    for k in range(K - 1, 0, -1):
        r0, _, r1 = G[k].shape
        C = G[k].reshape(r0, 2 * r1)
        Q, R = np.linalg.qr(C.T)                               # C = R^T Q^T
        m = Q.shape[1]
        G[k] = Q.T.reshape(m, 2, r1)
        p0 = G[k - 1].shape[0]
        G[k - 1] = np.einsum("aib,bc->aic", G[k - 1], R.T).reshape(p0, 2, m)
    norm = float(np.linalg.norm(G[0]))
    info["norm"] = norm
    if K == 1:
        info["ranks"] = [1, 1]
        return (G, info) if return_info else G
    tau = eps * norm / math.sqrt(K - 1)
    info["tau"] = tau
    for k in range(K - 1):
        r0, _, r1 = G[k].shape
        C = G[k].reshape(r0 * 2, r1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        r = truncation_rank(s, tau, max_rank)
        info["sv"].append(s.copy())
        if tau > 0:
            tails = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
            r_eps = truncation_rank(s, tau, 0)
            if max_rank <= 0 or r_eps <= max_rank:
                for t in (tails[r_eps], tails[r_eps - 1]):
                    info["margin"] = min(info["margin"], abs(t - tau * tau) / (tau * tau))
        U = U[:, :r].copy()
        Vt = Vt[:r].copy()
        U, Vt = _gauge(U, Vt)
        G[k] = U.reshape(r0, 2, r)
        SV = s[:r, None] * Vt
        q0, _, q1 = G[k + 1].shape
        G[k + 1] = (SV @ G[k + 1].reshape(q0, 2 * q1)).reshape(r, 2, q1)
    info["ranks"] = tt_ranks(G)
    return (G, info) if return_info else G


def tt_from_cores_sum(a_cores, b_cores):
    """Exact TT of ``full(a) + full(b)`` with ranks ``r_a + r_b`` (block cores).

    Used by tests: rounding a redundant representation must recover the
    ranks of the summed tensor.
    """
    K = len(a_cores)
    out = []
    for k in range(K):
        A, B = a_cores[k], b_cores[k]
        if K == 1:
            out.append(A + B)
        elif k == 0:
            out.append(np.concatenate([A, B], axis=2))
        elif k == K - 1:
            out.append(np.concatenate([A, B], axis=0))
        else:
            C = np.zeros((A.shape[0] + B.shape[0], 2, A.shape[2] + B.shape[2]))
            C[: A.shape[0], :, : A.shape[2]] = A
            C[A.shape[0]:, :, A.shape[2]:] = B
            out.append(C)
    return out


def storage_count(ranks) -> int:
    """Number of stored core entries ``sum_k r_{k-1} * 2 * r_k``."""
    return int(sum(ranks[k] * 2 * ranks[k + 1] for k in range(len(ranks) - 1)))
