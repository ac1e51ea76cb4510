"""Tensor-train algebra in float64 (paper section 2).  Test infrastructure only.

Conventions
-----------
* A TT is a list of cores; core ``k`` (0-based here, ``k+1`` in the paper) is
  an array of shape ``(r_{k}, n_k, r_{k+1})`` with ``r_0 = r_m = 1``.
* Multi-indices are int arrays of shape ``(m, N)``.
* The left unfolding ``L(U)`` of a core ``U`` of shape ``(p1, p2, p3)`` has
  rows ``(j, x)`` with ``j`` slow and ``x`` fast, i.e. ``U.reshape(p1*p2, p3)``;
  the right unfolding ``R(U)`` is ``U.reshape(p1, p2*p3)`` (section 2.1, "Left
  and right unfoldings").  With this order the Kronecker factor
  ``(T^{<=i-1} kron I_{d_i})`` of Algorithm 1 acts on rows ``(x_{<i}, x_i)``,
  which is numpy's C order for the separation ``T^{<i>}``.
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

Cores = List[np.ndarray]

_CHUNK = 1 << 16


def ranks_of(cores: Sequence[np.ndarray]) -> List[int]:
    return [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]


def shape_of(cores: Sequence[np.ndarray]) -> List[int]:
    return [int(c.shape[1]) for c in cores]


def tt_eval(cores: Sequence[np.ndarray], idx: np.ndarray) -> np.ndarray:
    """Entries ``T(x) = T_1(x_1,:) T_2(:,x_2,:) ... T_m(:,x_m)`` at each column of ``idx``.

    Section 2.1, "TT-format" (the defining product of core slices).
    Pinned against a per-entry loop of explicit matrix products.
    """
    idx = np.asarray(idx)
    m = len(cores)
    n_obs = idx.shape[1]
    out = np.empty(n_obs, dtype=np.float64)
    for s in range(0, n_obs, _CHUNK):
        e = min(n_obs, s + _CHUNK)
        v = cores[0][0, idx[0, s:e], :]                      # (B, r_1)
        for k in range(1, m):
            sl = np.transpose(cores[k][:, idx[k, s:e], :], (1, 0, 2))  # (B, r_{k}, r_{k+1})
            v = np.einsum("na,nab->nb", v, sl)
        out[s:e] = v[:, 0]
    return out


def left_part(cores: Sequence[np.ndarray], i: int) -> np.ndarray:
    """The i-th left part ``T^{<=i}``, shape ``(n_1...n_i, r_i)`` (section 2.1).

    Built by ``T^{<=k} = (T^{<=k-1} kron I_{n_k}) L(T_k)`` with ``T^{<=0} = [1]``.
    """
    left = np.ones((1, 1))
    for k in range(i):
        c = cores[k]
        left = (left @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return left


def right_part(cores: Sequence[np.ndarray], i: int) -> np.ndarray:
    """The i-th right part ``T^{>=i}`` (1-based i), shape ``(r_{i-1}, n_i...n_m)``.

    Built by ``T^{>=k}(:, x_k...) = T_k(:,x_k,:) T^{>=k+1}`` with ``T^{>=m+1} = [1]``.
    """
    m = len(cores)
    right = np.ones((1, 1))
    for k in range(m - 1, i - 2, -1):
        c = cores[k]
        right = (c.reshape(-1, c.shape[2]) @ right).reshape(c.shape[0], -1)
    return right


def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense tensor of a TT (only for tiny shapes)."""
    m = len(cores)
    return left_part(cores, m).reshape(shape_of(cores))


def separation(x: np.ndarray, i: int) -> np.ndarray:
    """The i-th separation ``X^{<i>}``: reshape to ``(n_1...n_i, n_{i+1}...n_m)`` (section 2.1)."""
    rows = int(np.prod(x.shape[:i])) if i > 0 else 1
    return x.reshape(rows, -1)


def mode_unfolding(x: np.ndarray, i: int) -> np.ndarray:
    """Mode-i unfolding ``M_i(X)`` of size ``n_i x prod_{k != i} n_k`` (section 2.1)."""
    return np.moveaxis(x, i, 0).reshape(x.shape[i], -1)


def tt_svd_dense(x: np.ndarray, ranks: Sequence[int]) -> Cores:
    """Algorithm 1 (TT-SVD) applied to a dense tensor.

    For i = 1..m-1: ``L(T_i)`` = the top ``r_i`` left singular vectors of
    ``(T^{<=i-1} kron I_{d_i})^T X^{<i>}``; ``T^{<=i} = (T^{<=i-1} kron I) L(T_i)``;
    finally ``T_m = (T^{<=m-1})^T X^{<m-1>}``.  Singular vectors come from
    ``numpy.linalg.svd``.
    """
    shape = list(x.shape)
    m = len(shape)
    left = np.ones((1, 1))
    cores: Cores = []
    for i in range(m - 1):
        n_i = shape[i]
        xi = x.reshape(left.shape[0], n_i, -1)              # rows x_{<i} | x_i | rest
        mat = np.einsum("pj,pxr->jxr", left, xi).reshape(left.shape[1] * n_i, -1)
        u, _, _ = np.linalg.svd(mat, full_matrices=False)
        r_i = int(ranks[i + 1])
        if u.shape[1] < r_i:
            raise ValueError("target rank exceeds the rank of the separation matrix")
        lt = u[:, :r_i]
        core = lt.reshape(left.shape[1], n_i, r_i)
        cores.append(core)
        left = (left @ core.reshape(core.shape[0], -1)).reshape(-1, r_i)
    last = left.T @ x.reshape(left.shape[0], -1)               # (r_{m-1}, n_m)
    cores.append(last.reshape(last.shape[0], shape[-1], 1))
    return cores


def tt_round(cores: Sequence[np.ndarray], ranks: Sequence[int]) -> Cores:
    """Algorithm 1 applied to a tensor given in TT format (any ranks), without forming it.

    Because ``X^{<i>} = X^{<=i} X^{>=i+1}``, making the right parts row-orthonormal
    first (a right-to-left sweep of Householder QRs of ``R(C_k)^T``) leaves the
    left singular vectors of ``(T^{<=i-1} kron I)^T X^{<i>}`` equal to those of
    ``L(P_{i-1} C_i)``, where ``P_{i-1} = (T^{<=i-1})^T X^{<=i-1}`` is carried
    from step to step as ``Sigma V^T`` of the truncated SVD.  The final core is
    ``P_{m-1} C_m``, Algorithm 1's ``(T^{<=m-1})^T X^{<m-1>}``.
    Pinned against :func:`tt_svd_dense` on the dense tensor.
    """
    c = [np.array(a, dtype=np.float64, copy=True) for a in cores]
    m = len(c)
    for k in range(m - 1, 0, -1):
        ra, n, rb = c[k].shape
        q, r = np.linalg.qr(c[k].reshape(ra, n * rb).T)        # R(C_k)^T = Q R
        c[k] = q.T.reshape(q.shape[1], n, rb)
        prev = c[k - 1]
        c[k - 1] = (prev.reshape(-1, ra) @ r.T).reshape(prev.shape[0], prev.shape[1], q.shape[1])
    out: Cores = []
    carry = np.ones((1, 1))
    for i in range(m - 1):
        b = np.einsum("ja,axb->jxb", carry, c[i])
        rows = b.shape[0] * b.shape[1]
        u, s, vt = np.linalg.svd(b.reshape(rows, -1), full_matrices=False)
        r_i = int(ranks[i + 1])
        if u.shape[1] < r_i:
            raise ValueError("target rank exceeds the rank of the separation matrix")
        out.append(u[:, :r_i].reshape(b.shape[0], b.shape[1], r_i))
        carry = s[:r_i, None] * vt[:r_i]
    out.append(np.einsum("ja,axb->jxb", carry, c[m - 1]))
    return out


def tt_inner(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """Euclidean inner product of two TTs of the same shape, by contracting cores."""
    z = np.ones((1, 1))
    for ca, cb in zip(a, b):
        z = np.einsum("ab,axc,bxd->cd", z, ca, cb)
    return float(z[0, 0])


def tt_add(a: Sequence[np.ndarray], b: Sequence[np.ndarray], beta: float = 1.0) -> Cores:
    """TT of ``A + beta*B`` with block cores (ranks add)."""
    m = len(a)
    out: Cores = []
    for k in range(m):
        ca, cb = a[k], b[k]
        if k == 0:
            out.append(np.concatenate([ca, beta * cb], axis=2))
        elif k == m - 1:
            out.append(np.concatenate([ca, cb], axis=0))
        else:
            z = np.zeros((ca.shape[0] + cb.shape[0], ca.shape[1], ca.shape[2] + cb.shape[2]))
            z[: ca.shape[0], :, : ca.shape[2]] = ca
            z[ca.shape[0]:, :, ca.shape[2]:] = cb
            out.append(z)
    return out


def tt_norm(cores: Sequence[np.ndarray]) -> float:
    """Frobenius norm, computed as the norm of the last core after a left QR sweep.

    Orthogonalising first avoids the cancellation of the Gram formula, so the
    norm of a difference of nearly equal tensors is accurate.
    """
    c = [np.array(x, dtype=np.float64, copy=True) for x in cores]
    for k in range(len(c) - 1):
        ra, n, rb = c[k].shape
        _, r = np.linalg.qr(c[k].reshape(ra * n, rb))
        nxt = c[k + 1]
        c[k + 1] = (r @ nxt.reshape(rb, -1)).reshape(r.shape[0], nxt.shape[1], nxt.shape[2])
    return float(np.linalg.norm(c[-1]))


def tt_dist(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """``||A - B||_F`` for two TTs, through the difference TT."""
    return tt_norm(tt_add(a, b, -1.0))


def left_orthogonalize(cores: Sequence[np.ndarray]):
    """Left-orthogonal decomposition by a Householder QR sweep (section 2.1).

    ``L(C_{k-1} S_k) = Q R`` with ``diag(R) >= 0``; the core becomes ``Q`` and
    ``R`` is carried into the next core.  Returns the cores (the last one
    carries the whole norm) and the carried factors ``[R_1, ..., R_{m-1}]``.
    """
    c = [np.array(x, dtype=np.float64, copy=True) for x in cores]
    factors = []
    for k in range(len(c) - 1):
        ra, n, rb = c[k].shape
        q, r = np.linalg.qr(c[k].reshape(ra * n, rb))
        sg = np.sign(np.diag(r))
        sg[sg == 0] = 1.0
        q = q * sg[None, :]
        r = sg[:, None] * r
        c[k] = q.reshape(ra, n, q.shape[1])
        nxt = c[k + 1]
        c[k + 1] = (r @ nxt.reshape(rb, -1)).reshape(r.shape[0], nxt.shape[1], nxt.shape[2])
        factors.append(r)
    return c, factors


def manifold_dim(shape: Sequence[int], ranks: Sequence[int]) -> int:
    """``dim M_r = sum_k r_{k-1} d_k r_k - sum_{k=1}^{m-1} r_k^2`` (section 5, OS ratio)."""
    m = len(shape)
    return int(sum(ranks[k] * shape[k] * ranks[k + 1] for k in range(m)) - sum(ranks[k] ** 2 for k in range(1, m)))
