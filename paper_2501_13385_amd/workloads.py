"""Seeded synthetic inputs for low-TT-rank completion problems.

This module only draws random numbers.  It produces the ingredients of a
completion problem -- the cores of a ground-truth tensor train, an
observation set drawn uniformly without replacement, a standard-normal noise
vector and a perturbation of the truth that serves as the starting point --
and performs no tensor-train arithmetic at all.  The observed values
``y = T*(x) + noise`` are formed by the consumer: the tests form them with the
reference implementation, the benchmark with the library's own evaluator.

Shapes follow the paper's problem statement (section 1, the completion model;
section 2, the TT format): an order-``m`` tensor with mode sizes ``n_k`` and
TT ranks ``r_0 = 1, r_1, ..., r_{m-1}, r_m = 1``.  A core is stored as a
float64 array of shape ``(r_{k-1}, n_k, r_k)``.  Index sets are returned as
int32 arrays of shape ``(m, N)`` (one row per mode, structure of arrays).

All draws use numpy's PCG64 generator, so a seed fixes a problem exactly.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "make_rng",
    "sample_indices",
    "gaussian_cores",
    "smooth_cores",
    "perturb_cores",
    "problem",
    "named",
    "NAMED",
    "serving_mix",
    "sketch_gaussians",
]


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _numel(shape: Sequence[int]) -> int:
    return int(math.prod(int(s) for s in shape))


def _decode(lin: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    """Mixed-radix decode of linear indices, mode 1 slowest."""
    m = len(shape)
    out = np.empty((m, lin.shape[0]), dtype=np.int32)
    rest = lin.astype(np.int64, copy=True)
    for k in range(m - 1, -1, -1):
        out[k] = (rest % shape[k]).astype(np.int32)
        rest //= shape[k]
    return out


def sample_indices(shape: Sequence[int], n_obs: int, rng: np.random.Generator) -> np.ndarray:
    """``n_obs`` distinct multi-indices, uniform without replacement.

    Small index spaces use ``choice(..., replace=False)``; large ones draw
    i.i.d. uniform multi-indices and keep first occurrences until ``n_obs``
    distinct ones are found (the first ``n_obs`` distinct values of an i.i.d.
    uniform stream form a uniformly random subset).  Order is random.
    """
    shape = [int(s) for s in shape]
    total = _numel(shape)
    if n_obs < 0 or n_obs > total:
        raise ValueError(f"cannot draw {n_obs} distinct entries from {total}")
    if total <= (1 << 26):
        lin = rng.choice(total, size=n_obs, replace=False)
        return _decode(np.asarray(lin, dtype=np.int64), shape)
    m = len(shape)
    rows: List[np.ndarray] = []
    seen = None
    need = n_obs
    while need > 0:
        draw = max(1024, int(need * 1.1) + 16)
        cand = np.stack([rng.integers(0, shape[k], size=draw, dtype=np.int64) for k in range(m)], axis=0)
        if total < (1 << 62):
            key = np.zeros(draw, dtype=np.int64)
            for k in range(m):
                key = key * shape[k] + cand[k]
            keyv = key
        else:  # row view as a structured key
            keyv = np.ascontiguousarray(cand.T).view([("", np.int64)] * m).reshape(-1)
        _, first = np.unique(keyv, return_index=True)
        first.sort()
        keyv = keyv[first]
        cand = cand[:, first]
        if seen is not None:
            fresh = ~np.isin(keyv, seen)
            keyv = keyv[fresh]
            cand = cand[:, fresh]
        take = min(need, cand.shape[1])
        rows.append(cand[:, :take])
        seen = keyv[:take] if seen is None else np.concatenate([seen, keyv[:take]])
        need -= take
    return np.concatenate(rows, axis=1).astype(np.int32)


def gaussian_cores(shape: Sequence[int], ranks: Sequence[int], rng: np.random.Generator,
                   std: Optional[Sequence[float]] = None) -> List[np.ndarray]:
    """I.i.d. normal cores; ``std[k]`` is the entry standard deviation of core k."""
    m = len(shape)
    if std is None:
        std = [1.0] * m
    return [rng.standard_normal((ranks[k], shape[k], ranks[k + 1])) * float(std[k]) for k in range(m)]


def unit_norm_std(shape: Sequence[int], ranks: Sequence[int]) -> List[float]:
    """Equal per-core standard deviations giving E||T||_F^2 = 1 for Gaussian cores.

    For independent zero-mean cores with entry variance s_k^2 one has
    E[T(x)^2] = prod_k s_k^2 * prod_{k=1}^{m-1} r_k, hence
    E||T||_F^2 = d* prod_k s_k^2 prod r_k.  This is a statement about the
    distribution, not a computation on the drawn cores.
    """
    m = len(shape)
    dstar = float(_numel(shape))
    prod_r = float(math.prod(ranks[1:m]))
    var = (dstar * prod_r) ** (-1.0 / m)
    return [math.sqrt(var)] * m


def smooth_cores(shape: Sequence[int], ranks: Sequence[int], rng: np.random.Generator,
                 terms: int = 8, max_freq: float = 3.0, perturb: float = 0.01) -> List[np.ndarray]:
    """Cores whose mode-index profile is a sum of random low-frequency cosines.

    Each entry ``T_k(a, :, b)`` is ``sum_q A_q cos(2 pi f_q x / n_k + phi_q)``
    with ``f_q ~ U[0, max_freq]``, ``phi_q ~ U[0, 2 pi)``, ``A_q ~ N(0, 1/terms)``,
    drawn independently per ``(k, a, b, q)``; then ``perturb * rms * N(0,1)`` is
    added to every core entry (the tensor stays exactly of TT rank ``ranks``).
    """
    cores = []
    for k in range(len(shape)):
        ra, n, rb = ranks[k], shape[k], ranks[k + 1]
        f = rng.uniform(0.0, max_freq, size=(ra, rb, terms))
        phi = rng.uniform(0.0, 2 * math.pi, size=(ra, rb, terms))
        amp = rng.standard_normal((ra, rb, terms)) / math.sqrt(terms)
        x = np.arange(n, dtype=np.float64)
        prof = (amp[:, :, :, None] * np.cos(2 * math.pi * f[:, :, :, None] * x / n + phi[:, :, :, None])).sum(axis=2)
        core = np.transpose(prof, (0, 2, 1)).copy()  # (ra, n, rb)
        rms = math.sqrt(float(np.mean(core * core)))
        core += perturb * rms * rng.standard_normal(core.shape)
        cores.append(core)
    return cores


def perturb_cores(cores: Sequence[np.ndarray], rel: float, rng: np.random.Generator) -> List[np.ndarray]:
    """Starting point: each core plus ``rel * rms(core) * N(0,1)`` noise.

    A perturbation of the cores keeps the TT ranks, so the result lies on the
    fixed-rank manifold, as the algorithm's initialisation requires.
    """
    out = []
    for c in cores:
        rms = math.sqrt(float(np.mean(c * c)))
        out.append(c + rel * rms * rng.standard_normal(c.shape))
    return out


@dataclasses.dataclass
class Problem:
    """Random ingredients of one completion problem (values not yet formed)."""

    name: str
    shape: List[int]
    ranks: List[int]
    truth: List[np.ndarray]          # ground-truth cores
    indices: np.ndarray              # int32 (m, N), distinct multi-indices
    noise: np.ndarray                # float64 (N,), standard normal (zero if noiseless)
    noise_std: float                 # absolute standard deviation to multiply ``noise`` by
    init: List[np.ndarray]           # starting cores (perturbed truth)
    stop_rule: str = "residual"      # "residual" | "change" | "error"
    tol: float = 1e-10
    max_iter: int = 500
    precision: str = "fp64"          # "fp64" | "mixed"
    step: float = 1.0                # step constant c in alpha = c * sqrt(eps) / p
    seed: int = 0

    @property
    def order(self) -> int:
        return len(self.shape)

    @property
    def n_obs(self) -> int:
        return int(self.indices.shape[1])

    @property
    def dstar(self) -> float:
        return float(math.prod(float(s) for s in self.shape))


def feasible_ranks(shape: Sequence[int], r: int) -> List[int]:
    """Interior ranks ``min(r, prod n_{<=k}, prod n_{>k})`` with r_0 = r_m = 1."""
    m = len(shape)
    out = [1]
    for k in range(1, m):
        left = math.prod(shape[:k])
        right = math.prod(shape[k:])
        out.append(int(min(r, left, right)))
    out.append(1)
    return out


def problem(shape: Sequence[int], ranks: Sequence[int], n_obs: int, seed: int, *,
            name: str = "custom", truth_kind: str = "gaussian", noise_rel: float = 0.0,
            init_rel: float = 0.1, stop_rule: str = "residual", tol: float = 1e-10,
            max_iter: int = 500, precision: str = "fp64", step: float = 1.0,
            core_std: Optional[Sequence[float]] = None) -> Problem:
    """Draw one problem.

    ``truth_kind``: ``gaussian`` (i.i.d. normal cores with ``core_std``, default
    unit variance), ``unit`` (Gaussian with equal variances giving unit
    expected Frobenius norm) or ``smooth`` (cosine profiles, see
    :func:`smooth_cores`).  ``noise_rel`` scales a standard-normal noise vector
    by ``noise_rel * sqrt(E||T*||^2 / d*)`` (the expected RMS entry), evaluated
    from the distribution, not the drawn cores.
    """
    shape = [int(s) for s in shape]
    ranks = [int(r) for r in ranks]
    rng = make_rng(seed)
    if truth_kind == "gaussian":
        truth = gaussian_cores(shape, ranks, rng, core_std)
        std = core_std if core_std is not None else [1.0] * len(shape)
        exp_sq = _numel(shape) * math.prod(s * s for s in std) * math.prod(ranks[1:-1])
    elif truth_kind == "unit":
        truth = gaussian_cores(shape, ranks, rng, unit_norm_std(shape, ranks))
        exp_sq = 1.0
    elif truth_kind == "smooth":
        truth = smooth_cores(shape, ranks, rng)
        exp_sq = float("nan")
    else:
        raise ValueError(truth_kind)
    idx = sample_indices(shape, n_obs, rng)
    noise = rng.standard_normal(n_obs) if noise_rel > 0 else np.zeros(n_obs)
    noise_std = noise_rel * math.sqrt(exp_sq / _numel(shape)) if noise_rel > 0 else 0.0
    init = perturb_cores(truth, init_rel, rng)
    return Problem(name=name, shape=shape, ranks=ranks, truth=truth, indices=idx, noise=noise,
                   noise_std=noise_std, init=init, stop_rule=stop_rule, tol=tol,
                   max_iter=max_iter, precision=precision, step=step, seed=seed)


def _c1(seed: int = 0) -> Problem:
    # order 4, n = 10, ranks (1,2,2,2,1), 30% of 10^4 entries, noiseless
    return problem([10] * 4, [1, 2, 2, 2, 1], 3000, seed, name="c1_m4_n10_r2",
                   truth_kind="gaussian", stop_rule="residual", tol=1e-10, max_iter=500)


def _c2(seed: int = 0) -> Problem:
    # order 3, n = 400, ranks (1,10,10,1), 1% sampling, noise 1e-3 x RMS entry
    return problem([400] * 3, [1, 10, 10, 1], 640_000, seed, name="c2_m3_n400_r10",
                   truth_kind="unit", noise_rel=1e-3, stop_rule="change", tol=1e-6,
                   max_iter=500, init_rel=0.1)


def _c3(seed: int = 0) -> Problem:
    # 256 x 256 x 128, ranks (1,16,16,1), smooth cores, 5% observed, noiseless
    shape = [256, 256, 128]
    return problem(shape, [1, 16, 16, 1], int(0.05 * _numel(shape)), seed, name="c3_img_256x256x128_r16",
                   truth_kind="smooth", stop_rule="error", tol=1e-6, max_iter=500,
                   precision="mixed", init_rel=0.1)


def _c4(seed: int = 0) -> Problem:
    # order 14, n = 4, interior ranks 8 clipped at the boundaries, 2M samples
    shape = [4] * 14
    ranks = feasible_ranks(shape, 8)
    std = [1.0 / math.sqrt(ranks[k + 1]) for k in range(14)]
    return problem(shape, ranks, 2_000_000, seed, name="c4_mps_m14_n4_r8", truth_kind="gaussian",
                   core_std=std, stop_rule="error", tol=1e-6, max_iter=500, precision="mixed",
                   init_rel=0.1)


def _hbm3(seed: int = 0) -> Problem:
    # order 3, n = 1000, ranks (1,2,2,1), 50,000,000 samples (5%), noiseless:
    # 20 bytes and ~36 flop per sample, a shape where the sampled pass is bound
    # by memory bandwidth rather than arithmetic
    return problem([1000] * 3, [1, 2, 2, 1], 50_000_000, seed, name="hbm3_m3_n1000_r2", truth_kind="unit",
                   stop_rule="error", tol=1e-6, max_iter=500, init_rel=0.1)


def _c2_small(seed: int = 0) -> Problem:
    # a C2-shaped case small enough for the reference to iterate in seconds
    return problem([40, 36, 44], [1, 4, 4, 1], 6000, seed, name="c2_small_m3_r4",
                   truth_kind="unit", noise_rel=1e-3, stop_rule="change", tol=1e-6, max_iter=200,
                   init_rel=0.1)


NAMED = {
    "c1": _c1,
    "c2": _c2,
    "c3": _c3,
    "c4": _c4,
    "c2_small": _c2_small,
    "hbm3": _hbm3,
}


def named(name: str, seed: int = 0) -> Problem:
    return NAMED[name](seed)


def serving_mix(n_requests: int = 512, seed: int = 0, *, max_obs: int = 4_194_304,
                min_os: float = 6.0, rate: float = 1000.0) -> List[dict]:
    """Request stream for the serving workload.

    Each request draws order m in {3,4,5,8}, one mode size n in [20, 300] for
    all modes, a rank r in {2,4,8,16} (clipped to feasibility) and a sampling
    ratio in [0.5%, 10%]; the observation count is capped at ``max_obs`` and
    redrawn (counted) when the oversampling ratio |Omega| / dim M_r would fall
    below ``min_os``.  Arrivals form a Poisson process with rate ``rate`` per
    second.  Returns dicts with ``shape``, ``ranks``, ``n_obs``, ``seed`` and
    ``arrival`` (seconds); the problem itself is drawn later with
    :func:`problem` from ``seed``.
    """
    rng = make_rng(seed)
    reqs = []
    t = 0.0
    redraws = 0
    while len(reqs) < n_requests:
        m = int(rng.choice([3, 4, 5, 8]))
        n = int(rng.integers(20, 301))
        r = int(rng.choice([2, 4, 8, 16]))
        ratio = float(rng.uniform(0.005, 0.10))
        shape = [n] * m
        ranks = feasible_ranks(shape, r)
        dim = sum(ranks[k] * shape[k] * ranks[k + 1] for k in range(m)) - sum(ranks[k] ** 2 for k in range(1, m))
        n_obs = int(min(math.floor(ratio * float(n) ** m), max_obs))
        if n_obs < min_os * dim:
            redraws += 1
            continue
        t += float(rng.exponential(1.0 / rate))
        reqs.append({"shape": shape, "ranks": ranks, "n_obs": n_obs,
                     "seed": int(rng.integers(0, 2**31 - 1)), "arrival": t, "redraws": redraws})
    return reqs


def random_mps(n_sites: int, bond: int, rng: np.random.Generator, local: int = 2) -> List[np.ndarray]:
    """Random matrix product state for the quantum-state-tomography workload (section
    5.3): complex cores ``U_k`` of shape ``(s_{k-1}, local, s_k)`` with i.i.d. standard
    complex normal entries, ``s_k = min(bond, local^k, local^(n-k))``, ``s_0 = s_n = 1``."""
    out = []
    for k in range(n_sites):
        sl = min(bond, local ** k, local ** (n_sites - k))
        sr = min(bond, local ** (k + 1), local ** (n_sites - k - 1))
        re = rng.standard_normal((sl, local, sr))
        im = rng.standard_normal((sl, local, sr))
        out.append((re + 1j * im) / math.sqrt(2.0))
    return out


def sketch_gaussians(shape: Sequence[int], sketch: int, rng: np.random.Generator) -> List[np.ndarray]:
    """Standard-normal test matrices for the sketched spectral initialisation.

    For every split i = 0..m-2 (0-based) and every later mode k = i+1..m-1 one
    ``(n_k, sketch)`` matrix, in that order (split-major).  Returned as a flat
    list; ``numpy.concatenate([g.ravel() for g in ...])`` is the packed layout
    the library takes.
    """
    m = len(shape)
    out: List[np.ndarray] = []
    for i in range(m - 1):
        for k in range(i + 1, m):
            out.append(rng.standard_normal((int(shape[k]), int(sketch))))
    return out
