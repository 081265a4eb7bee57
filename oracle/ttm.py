"""TT-SVD and max-rank TT-RSVD on tensors with mode sizes other than 2, in float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5 notes that the randomised variant (modification (2): the SVD of
Algorithm 1 replaced by Algorithms 4 and 5 with ``ell = R_max + p``
columns) pays off for larger mode sizes ``M_k``, where the unfoldings have
``m_k = M_k r_{k-1}`` rows, and times a ``K = 8``, ``M_k = 10`` tensor of
uniform entries.  These functions state both sweeps for a tensor with mode
sizes ``modes = (M_1, ..., M_K)``:

* the tensor is the vector ``a`` with index ``i = i_1 + M_1 (i_2 + M_2 (...))``
  (first mode fastest, as the QTT map of Section 5);
* step ``k`` unfolds the remainder column-major into ``A_k`` of shape
  ``(M_k r_{k-1}) x (prod_{j>k} M_j)`` and keeps ``U_k[:, :r_k]`` as core
  ``k`` of shape ``(r_{k-1}, M_k, r_k)``; the remainder is ``Sigma V^T``;
* the rank is Algorithm 1's rule on the singular values (tolerance
  ``tau = eps ||a|| / sqrt(K-1)``, then the cap ``R_max``), as in
  :mod:`oracle.tt`;
* the randomised step draws ``Omega`` (``n_k x ell``) from
  :func:`oracle.rsvd.gaussian_matrix` with ``step = k`` and takes the rank
  from the singular values of ``B = Q^T A``; where ``min(m_k, n_k) <= R_max
  + p`` it reverts to the exact SVD, as Section 5 prescribes.
"""

from __future__ import annotations

import math

import numpy as np

from . import rsvd, tt


def _check(a, modes):
    v = np.asarray(a, dtype=np.float64).ravel(order="F")
    if int(np.prod(modes)) != v.size:
        raise ValueError("the mode sizes do not match the number of entries")
    return v


def tt_svd_modes(a, modes, eps: float, max_rank: int = 0, return_info: bool = False,
                 method: str = "svd", oversample: int = 10, seed: int = 0):
    """Algorithm 1 on the tensor ``a`` with mode sizes ``modes``.

    ``method="svd"``: exact truncated SVDs (modification (1) through
    ``max_rank``); ``method="rsvd"``: the max-rank TT-RSVD of modification (2)
    with ``ell = max_rank + oversample`` (``max_rank`` must be positive).
    Returns the cores (and, with ``return_info``, the threshold, ranks and
    the singular values each step's rule saw).
    """
    modes = [int(m) for m in modes]
    K = len(modes)
    v = _check(a, modes)
    norm = float(np.linalg.norm(v))
    info = {"norm": norm, "ranks": [1], "sv": [], "exact_steps": []}
    if method == "rsvd" and max_rank <= 0:
        raise ValueError("the randomised sweep needs a rank cap")
    if K == 1:
        cores = [v.reshape(1, modes[0], 1).copy()]
        info["ranks"].append(1)
        info["tau"] = 0.0
        return (cores, info) if return_info else cores
    tau = eps * norm / math.sqrt(K - 1)
    info["tau"] = tau
    cores = []
    r_prev = 1
    rem = v
    for k in range(1, K):
        m = modes[k - 1] * r_prev
        A = rem.reshape((m, -1), order="F")
        ell = max_rank + oversample
        if method == "rsvd" and min(A.shape) > ell:
            omega = rsvd.gaussian_matrix(A.shape[1], ell, k, seed)
            Q = rsvd.range_finder(A, omega)
            U, s, Vt = rsvd.rsvd(A, Q)
            info["exact_steps"].append(False)
        else:
            U, s, Vt = np.linalg.svd(A, full_matrices=False)
            info["exact_steps"].append(True)
        r = tt.truncation_rank(s, tau, max_rank)
        info["sv"].append(s.copy())
        U, Vt = tt._gauge(U[:, :r].copy(), Vt[:r, :].copy())
        cores.append(U.reshape((r_prev, modes[k - 1], r), order="F"))
        rem = (s[:r, None] * Vt).ravel(order="F")
        info["ranks"].append(r)
        r_prev = r
    cores.append(rem.reshape((r_prev, modes[K - 1], 1), order="F"))
    info["ranks"].append(1)
    return (cores, info) if return_info else cores


def tt_full_modes(cores) -> np.ndarray:
    """Algorithm 3 for general mode sizes: the entries in the index order above."""
    A = np.asarray(cores[0], dtype=np.float64)
    A = A.reshape((-1, A.shape[2]), order="F")
    for G in cores[1:]:
        r0, M, r1 = G.shape
        A = A.reshape((-1, r0), order="F") @ np.asarray(G, dtype=np.float64).reshape(
            (r0, M * r1), order="F")
        A = A.reshape((-1, r1), order="F")
    return A.reshape(-1, order="F")


def tt_entry_modes(cores, idx: int) -> float:
    """One entry as the product of the core slices picked by the digits of ``idx``."""
    row = np.ones((1, 1))
    for G in cores:
        M = G.shape[1]
        row = row @ G[:, idx % M, :]
        idx //= M
    return float(row[0, 0])
