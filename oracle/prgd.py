"""Preconditioned Riemannian gradient descent (PRGD) in float64.  Test infrastructure only.

This follows the paper's section 3 and Algorithm 2 step by step, with the
trimming step skipped (section 3.2.2 notes that the method behaves the same
without it).  Readings of passages the paper leaves open (all listed in the
design notes of the repository):

* ``eps_l = ||G_l||_vee^2`` (the choice made in the convergence proof,
  Appendix B), i.e. the largest squared mode-slice norm of the sparse
  gradient; a fixed ``eps`` may be given instead.
* The metric is ``W = x_i G_{l,i}^{1/(2m)}``, so ``W^{1/2}`` scales core ``i``'s
  mode index by ``g_i^{1/(4m)}`` (Proposition 1, Lemma 3), ``m`` the tensor order.
* Step policies: ``theory`` ``alpha_l = c * eps_l^{1/2} / p`` (Theorem 1 with
  ``c = 1.001``), ``const`` (fixed ``alpha`` with fixed ``eps``), ``adaptive``
  (eq. "PRGD stepsize"); ``p = |Omega| / d*``.
* The left-orthogonal decomposition of ``W^{1/2} T`` (section 3.3) is taken by
  a Householder QR sweep; the tangent projection is the closed form of
  Lemma 3, evaluated with a second pass over the samples in the weighted
  ("hat") space.
* The retraction is Algorithm 1 applied to ``W_l`` given in block-TT form.
* Observed values ``y`` stand in for ``T*`` on ``Omega`` (with noise they differ).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg

from . import tt

Cores = List[np.ndarray]

_CHUNK = 1 << 15


# ----------------------------------------------------------------------------
# sampled quantities
# ----------------------------------------------------------------------------

def residual(cores: Sequence[np.ndarray], idx: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Entries of ``G_l = P_Omega(T_l - T*)`` on Omega (Algorithm 2, first step)."""
    return tt.tt_eval(cores, idx) - np.asarray(y, dtype=np.float64)


def slice_norms(idx: np.ndarray, r: np.ndarray, shape: Sequence[int]) -> List[np.ndarray]:
    """``s_i(k) = ||M_i(G)(k,:)||_2^2``, the squared mode-i slice norms of the sparse gradient.

    Section 3.2.1: the diagonal of ``M_i(G_l) M_i(G_l)^T``.  For a tensor that is
    zero off Omega this is the sum of ``R_j^2`` over samples with ``x_i = k``.
    """
    rr = r * r
    return [np.bincount(idx[i], weights=rr, minlength=shape[i]).astype(np.float64) for i in range(len(shape))]


def eps_vee(s: Sequence[np.ndarray]) -> float:
    """``||G_l||_vee^2 = max_i max_k ||M_i(G_l)(k,:)||^2`` (Notations)."""
    return float(max(np.max(x) if x.size else 0.0 for x in s))


def core_gradient(cores: Sequence[np.ndarray], idx: np.ndarray, r: np.ndarray) -> Cores:
    """Euclidean gradient of ``f`` with respect to each core (chain rule on eq. "TT Core").

    ``df/dT_i(:, x_i, :) = sum_{j : x_i^{(j)} = x_i} R_j  (T^{<=i-1}(x_{<i}))^T (T^{>=i+1}(x_{>i}))^T``
    with ``f = 1/2 sum_j R_j^2``.  Pinned by central finite differences.
    """
    m = len(cores)
    grads = [np.zeros((c.shape[1], c.shape[0], c.shape[2])) for c in cores]   # (n, ra, rb)
    n_obs = idx.shape[1]
    for s in range(0, n_obs, _CHUNK):
        e = min(n_obs, s + _CHUNK)
        lv, rv = _interfaces(cores, idx[:, s:e])
        for i in range(m):
            outer = r[s:e, None, None] * lv[i][:, :, None] * rv[i + 2][:, None, :]
            np.add.at(grads[i], idx[i, s:e], outer)
    return [np.transpose(g, (1, 0, 2)).copy() for g in grads]


def _interfaces(cores: Sequence[np.ndarray], idx: np.ndarray):
    """Per-sample left parts ``lv[k] = T^{<=k}(x_{<=k})`` (k = 0..m) and right parts
    ``rv[k] = T^{>=k}(x_{>=k})`` (k = 1..m+1, 1-based), section 2.1."""
    m = len(cores)
    b = idx.shape[1]
    lv = [np.ones((b, 1))]
    for k in range(m):
        sl = np.transpose(cores[k][:, idx[k], :], (1, 0, 2))
        lv.append(np.einsum("na,nab->nb", lv[-1], sl))
    rv: List[Optional[np.ndarray]] = [None] * (m + 2)
    rv[m + 1] = np.ones((b, 1))
    for k in range(m, 0, -1):
        sl = np.transpose(cores[k - 1][:, idx[k - 1], :], (1, 0, 2))
        rv[k] = np.einsum("nab,nb->na", sl, rv[k + 1])
    return lv, rv


# ----------------------------------------------------------------------------
# the preconditioned tangent projection (section 3.3, Lemma 3)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Direction:
    """``xi = P~_T W^{-1} G = sum_i [T~_1, ..., A_i, ..., T~_m]`` and its ingredients."""

    base: Cores        # T~_i = T^_i x_2 G_i^{-1/(4m)}: the new left-orthogonal decomposition
    comps: Cores       # A_i = A^_i x_2 G_i^{-1/(4m)}
    hat_base: Cores    # T^_i: left-orthogonal decomposition of W^{1/2} T
    hat_comps: Cores   # A^_i from eq. "tsp in nm"
    g: List[np.ndarray]
    eps: float


def metric_diagonals(s: Sequence[np.ndarray], eps: float) -> List[np.ndarray]:
    """Diagonals of ``G_{l,i} = eps I + diag(M_i(G_l) M_i(G_l)^T)`` (section 3.2.1)."""
    return [eps + x for x in s]


def scale_mode(core: np.ndarray, w: np.ndarray) -> np.ndarray:
    """``core x_2 diag(w)``: scale the mode index of a core (Proposition 1)."""
    return core * w[None, :, None]


def tangent_direction(cores: Sequence[np.ndarray], idx: np.ndarray, r: np.ndarray,
                      eps: Optional[float] = None, metric: str = "data") -> Direction:
    """The Riemannian gradient under the data-driven metric, ``P~_T W^{-1} G_l``.

    Steps (section 3.3 and Lemma 3):

    1. ``g_i = eps + s_i`` (metric diagonals); ``eps = ||G||_vee^2`` unless given.
       With ``metric="euclidean"`` every ``g_i`` is 1, so ``W`` is the identity and
       the direction is the Euclidean tangent projection of ``G`` used by RGD
       (section 3.1).
    2. ``W^{1/2} T = [T_1 x_2 g_1^{1/(4m)}, ...]`` (Proposition 1), then its
       left-orthogonal decomposition ``[T^_1, ..., T^_m]`` by Householder QR.
    3. ``W^{-1/2} G`` on Omega: ``R_j prod_k g_k(x_k)^{-1/(4m)}``.
    4. ``B_i = (T^{<=i-1} kron I)^T (W^{-1/2}G)^{<i>} (T^{>=i+1})^T`` by a pass over
       the samples using the hat cores' left/right parts.
    5. ``L(A^_i) = (I - L(T^_i) L(T^_i)^T) L(B_i) (T^{>=i+1} T^{>=i+1,T})^{-1}`` for
       ``i < m`` (Cholesky solve), ``L(A^_m) = L(B_m)`` (eq. "tsp in nm").
    6. ``A_i = A^_i x_2 g_i^{-1/(4m)}``, ``T~_i = T^_i x_2 g_i^{-1/(4m)}`` (eq. "new
       left orthogonal").
    """
    m = len(cores)
    shape = tt.shape_of(cores)
    s = slice_norms(idx, r, shape)
    if eps is None:
        eps = eps_vee(s)
    if metric == "euclidean":
        g = [np.ones_like(x) for x in s]
    elif metric == "data":
        g = metric_diagonals(s, eps)
    else:
        raise ValueError(metric)
    e = 1.0 / (4.0 * m)
    shat = [scale_mode(cores[k], g[k] ** e) for k in range(m)]
    that, _ = tt.left_orthogonalize(shat)

    # right Grams H^_k = T^{>=k} T^{>=k,T}, k = m+1 .. 2 (1-based), by the core recursion
    hgram: List[Optional[np.ndarray]] = [None] * (m + 2)
    hgram[m + 1] = np.ones((1, 1))
    for k in range(m, 1, -1):
        c = that[k - 1]
        hgram[k] = np.einsum("axb,bc,dxc->ad", c, hgram[k + 1], c)

    ghat = r.copy()
    for k in range(m):
        ghat = ghat * g[k][idx[k]] ** (-e)

    bacc = [np.zeros((c.shape[1], c.shape[0], c.shape[2])) for c in that]
    n_obs = idx.shape[1]
    for st in range(0, n_obs, _CHUNK):
        en = min(n_obs, st + _CHUNK)
        lv, rv = _interfaces(that, idx[:, st:en])
        for i in range(m):
            outer = ghat[st:en, None, None] * lv[i][:, :, None] * rv[i + 2][:, None, :]
            np.add.at(bacc[i], idx[i, st:en], outer)
    bmat = [np.transpose(b, (1, 0, 2)) for b in bacc]

    hat_comps: Cores = []
    for i in range(m):
        ra, n, rb = that[i].shape
        lb = bmat[i].reshape(ra * n, rb)
        if i < m - 1:
            lt = that[i].reshape(ra * n, rb)
            z = lb - lt @ (lt.T @ lb)
            cf = scipy.linalg.cho_factor(hgram[i + 2])
            z = scipy.linalg.cho_solve(cf, z.T).T
        else:
            z = lb
        hat_comps.append(z.reshape(ra, n, rb))
    base = [scale_mode(that[k], g[k] ** (-e)) for k in range(m)]
    comps = [scale_mode(hat_comps[k], g[k] ** (-e)) for k in range(m)]
    return Direction(base=base, comps=comps, hat_base=that, hat_comps=hat_comps, g=g, eps=float(eps))


def tangent_tt(base: Sequence[np.ndarray], comps: Sequence[np.ndarray], alpha: float = 1.0,
               add_base: bool = False) -> Cores:
    """Block TT of ``B + alpha * sum_i [B_1..C_i..B_m]`` (``add_base``) or of the sum alone.

    Block cores ``[X_1, B_1]``, ``[[B_k, 0], [X_k, B_k]]`` and ``[[B_m], [X_m (+ B_m)]]``
    with ``X_i = alpha C_i``; their product is the sum of the m terms with one
    core replaced (section 3.3, tangent parameterisation).
    """
    m = len(base)
    out: Cores = []
    for k in range(m):
        b = base[k]
        x = alpha * comps[k]
        ra, n, rb = b.shape
        if m == 1:
            out.append(x + b if add_base else x)
        elif k == 0:
            out.append(np.concatenate([x, b], axis=2))
        elif k == m - 1:
            out.append(np.concatenate([b, x + b if add_base else x], axis=0))
        else:
            z = np.zeros((2 * ra, n, 2 * rb))
            z[:ra, :, :rb] = b
            z[ra:, :, :rb] = x
            z[ra:, :, rb:] = b
            out.append(z)
    return out


# ----------------------------------------------------------------------------
# step sizes (section 3.2.2, Theorem 1)
# ----------------------------------------------------------------------------

def sampling_ratio(n_obs: int, shape: Sequence[int]) -> float:
    """``p = |Omega| / d*`` (``d* = d_1 ... d_m``), computed in floating point."""
    return float(n_obs) / math.prod(float(s) for s in shape)


def step_theory(c: float, eps: float, p: float) -> float:
    """``alpha_l = c * eps_l^{1/2} / p``; Theorem 1 uses ``c = 1.001``."""
    return c * math.sqrt(eps) / p


def step_adaptive(d: Direction, idx: np.ndarray) -> float:
    """Steepest step ``||xi||_W^2 / ||P_Omega xi||_F^2`` (eq. "PRGD stepsize").

    ``||xi||_W^2 = ||W^{1/2} xi||_F^2`` and ``W^{1/2} xi = sum_i [T^_1..A^_i..T^_m]``
    (Lemma 3), whose norm is taken in TT form; the denominator evaluates ``xi`` on Omega.
    """
    num = tt.tt_norm(tangent_tt(d.hat_base, d.hat_comps)) ** 2
    xi_vals = tt.tt_eval(tangent_tt(d.base, d.comps), idx)
    den = float(np.dot(xi_vals, xi_vals))
    return num / den if den > 0 else 0.0


# ----------------------------------------------------------------------------
# Algorithm 2
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Policy:
    step_rule: str = "theory"        # "theory" | "const" | "adaptive"
    c: float = 1.001                 # constant of the theory step
    alpha: float = 0.0               # fixed step for "const"
    eps: Optional[float] = None      # fixed eps (required by "const"); None: eps_l = ||G_l||_vee^2
    stop_rule: str = "residual"      # "residual" | "change" | "error"
    tol: float = 1e-10
    max_iter: int = 500
    metric: str = "data"             # "data" (PRGD, section 3.2.1) | "euclidean" (RGD, section 3.1)


@dataclasses.dataclass
class Result:
    cores: Cores
    iterations: int
    status: str                      # "converged" | "max_iter" | "exact"
    history: List[dict]
    iterates: Optional[List[Cores]] = None


def prgd_step(cores: Sequence[np.ndarray], idx: np.ndarray, y: np.ndarray, policy: Policy,
              ranks: Sequence[int]):
    """One iteration ``T_l -> T_{l+1}`` of Algorithm 2 (trimming skipped).

    Returns ``(T_{l+1} or None if G_l = 0, info)``.
    """
    shape = tt.shape_of(cores)
    r = residual(cores, idx, y)
    info = {"res_norm": float(np.linalg.norm(r))}
    s = slice_norms(idx, r, shape)
    eps = eps_vee(s) if policy.eps is None else float(policy.eps)
    info["eps"] = eps
    if eps_vee(s) == 0.0:
        return None, info
    euclid = policy.metric == "euclidean"
    if euclid:
        eps = 1.0        # the Euclidean metric has no eps
        info["eps"] = eps
    d = tangent_direction(cores, idx, r, eps, policy.metric)
    p = sampling_ratio(idx.shape[1], shape)
    if policy.step_rule == "theory":
        # RGD's constant step in the same units: c / p (eps = 1)
        alpha = step_theory(policy.c, eps, p)
    elif policy.step_rule == "const":
        alpha = float(policy.alpha)
    elif policy.step_rule == "adaptive":
        alpha = step_adaptive(d, idx)
    else:
        raise ValueError(policy.step_rule)
    info["alpha"] = alpha
    w = tangent_tt(d.base, d.comps, -alpha, add_base=True)     # W_l = T_l - alpha xi
    return tt.tt_round(w, ranks), info


def prgd(init: Sequence[np.ndarray], idx: np.ndarray, y: np.ndarray, policy: Policy,
         truth: Optional[Sequence[np.ndarray]] = None, keep_iterates: bool = False,
         callback: Optional[Callable[[int, Cores, dict], None]] = None) -> Result:
    """Run Algorithm 2 from ``init`` until the stopping rule holds or ``max_iter`` iterations.

    Stopping rules: ``residual`` -- ``||P_Omega T_l - y|| / ||y|| <= tol`` tested on
    ``T_l`` before iteration l; ``change`` -- ``||T_{l+1} - T_l||_F <= tol * max(1,
    ||T_l||_F)`` (section 5.1, noise experiment); ``error`` -- ``||T_{l+1} - T*||_F /
    ||T*||_F <= tol`` (section 5.1, needs ``truth``).
    """
    idx = np.asarray(idx)
    y = np.asarray(y, dtype=np.float64)
    ranks = tt.ranks_of(init)
    cores = [np.array(c, dtype=np.float64, copy=True) for c in init]
    ynorm = float(np.linalg.norm(y))
    tnorm = tt.tt_norm(truth) if truth is not None else None
    hist: List[dict] = []
    iterates = [cores] if keep_iterates else None
    status = "max_iter"
    it = 0
    while it < policy.max_iter:
        new, info = prgd_step(cores, idx, y, policy, ranks)
        info["iter"] = it
        info["rel_res"] = info["res_norm"] / ynorm if ynorm > 0 else info["res_norm"]
        if policy.stop_rule == "residual" and info["rel_res"] <= policy.tol:
            hist.append(info)
            status = "converged"
            break
        if new is None:
            hist.append(info)
            status = "exact"
            break
        if policy.stop_rule == "change":
            info["rel_change"] = tt.tt_dist(new, cores) / max(1.0, tt.tt_norm(cores))
        cores = new
        it += 1
        if truth is not None:
            info["rel_err"] = tt.tt_dist(cores, truth) / tnorm
        hist.append(info)
        if keep_iterates:
            iterates.append(cores)
        if callback is not None:
            callback(it, cores, info)
        if policy.stop_rule == "change" and info["rel_change"] <= policy.tol:
            status = "converged"
            break
        if policy.stop_rule == "error" and info["rel_err"] <= policy.tol:
            status = "converged"
            break
    return Result(cores=cores, iterations=it, status=status, history=hist, iterates=iterates)


def spectral_init_dense(idx: np.ndarray, y: np.ndarray, shape: Sequence[int], ranks: Sequence[int]) -> Cores:
    """``T_0 = SVD^tt_r(P_Omega(y) / p)`` by Algorithm 1 on the dense tensor (tiny shapes)."""
    x = np.zeros(shape)
    x[tuple(idx)] = y
    return tt.tt_svd_dense(x / sampling_ratio(idx.shape[1], shape), ranks)


def spectral_init_sketch(idx: np.ndarray, y: np.ndarray, shape: Sequence[int], ranks: Sequence[int],
                         gauss: Sequence[np.ndarray]) -> Cores:
    """``T_0 ~ SVD^tt_r(P_Omega(y) / p)``: Algorithm 1 with every unfolding replaced by a sketch.

    Z = P_Omega(y) / p with p = |Omega| / d* (the spectral initialisation the
    convergence analysis assumes).  Algorithm 1 takes at split i the top r_i
    left singular vectors of the projected unfolding
    A_i = (T^{<=i-1} kron I_{n_i})^T Z^{<i>}, whose columns run over the later
    modes.  Here A_i is multiplied on the right by a random test matrix Psi_i
    whose row for the later indices (x_{i+1}, ..., x_m) is the elementwise
    product of the rows Gamma_{i,k}[x_k, :] of independent standard-normal
    matrices (one per later mode; E[Psi Psi^T] is a multiple of I), and the
    core is the top r_i left singular vectors of the sketch Y_i = A_i Psi_i.
    Y_i only needs the observed entries:
    Y_i[(a, x), c] = sum over samples with x_i = x of
    z_j ell_{i-1}(x^(j))[a] psi_i(x^(j))[c], with ell the interface of the
    cores already built.  The last core is A_m itself.

    ``gauss``: the matrices Gamma_{i,k} in split-major order (see
    ``workloads.sketch_gaussians``).  Plain float64: the sums run mode value by
    mode value over the matching samples; singular vectors from
    ``numpy.linalg.svd``.
    """
    shape = [int(s) for s in shape]
    m = len(shape)
    idx = np.asarray(idx, dtype=np.int64)
    n_obs = idx.shape[1]
    z = np.asarray(y, dtype=np.float64) / sampling_ratio(n_obs, shape)
    ell = np.ones((n_obs, 1))                     # ell_{i-1}(x^(j)), one row per sample
    cores: Cores = []
    g = 0
    for i in range(m - 1):
        r_prev, n_i, r_i = int(ranks[i]), shape[i], int(ranks[i + 1])
        psi = None
        for k in range(i + 1, m):
            rows = np.asarray(gauss[g])[idx[k]]       # Gamma_{i,k}[x_k(j), :]
            psi = rows if psi is None else psi * rows
            g += 1
        sketch = psi.shape[1]
        Y = np.zeros((r_prev, n_i, sketch))
        zl = z[:, None] * ell
        for x in range(n_i):                           # samples with x_i = x
            sel = idx[i] == x
            Y[:, x, :] = zl[sel].T @ psi[sel]
        ymat = Y.reshape(r_prev * n_i, sketch)
        u, sv, _ = np.linalg.svd(ymat, full_matrices=False)
        # Algorithm 1 keeps the top r_i left singular vectors; they are only
        # defined when the sketch has r_i singular values that float64 can tell
        # from zero.  Numerical rank in the usual sense: singular values above
        # max(rows, cols) * eps * sigma_1 (rounding of an SVD in float64).
        tol = max(ymat.shape) * np.finfo(np.float64).eps * (sv[0] if sv.size else 0.0)
        if u.shape[1] < r_i or not sv[r_i - 1] > tol:
            raise ValueError("sketch rank below the target rank")
        core = u[:, :r_i].reshape(r_prev, n_i, r_i)
        cores.append(core)
        ell = np.einsum("ja,ajb->jb", ell, core[:, idx[i], :])
    r_prev, n_m = int(ranks[m - 1]), shape[m - 1]
    last = np.zeros((r_prev, n_m))
    zl = z[:, None] * ell
    for x in range(n_m):
        last[:, x] = zl[idx[m - 1] == x].sum(axis=0)
    cores.append(last.reshape(r_prev, n_m, 1))
    return cores
