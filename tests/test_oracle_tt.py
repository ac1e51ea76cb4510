"""Pins for the reference TT algebra (oracle/tt.py) against brute force and closed forms."""

import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import tt
from paper_2501_13385_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_tt(shape, ranks, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((ranks[k], shape[k], ranks[k + 1])) for k in range(len(shape))]


def brute_entry(cores, x):
    """T(x) by an explicit left-to-right loop of matrix products."""
    v = np.eye(1)
    for k, c in enumerate(cores):
        v = v @ c[:, x[k], :]
    return v[0, 0]


def test_eval_matches_entrywise_products():
    shape, ranks = [3, 4, 2, 5], [1, 2, 3, 2, 1]
    cores = rand_tt(shape, ranks, 1)
    allx = np.array(list(itertools.product(*[range(n) for n in shape]))).T
    vals = tt.tt_eval(cores, allx)
    ref = np.array([brute_entry(cores, allx[:, j]) for j in range(allx.shape[1])])
    np.testing.assert_allclose(vals, ref, rtol=1e-13, atol=1e-13)
    full = tt.tt_full(cores)
    np.testing.assert_allclose(full[tuple(allx)], ref, rtol=1e-13, atol=1e-13)


def test_separation_factorises_into_left_and_right_parts():
    shape, ranks = [3, 4, 2, 5], [1, 2, 3, 2, 1]
    cores = rand_tt(shape, ranks, 2)
    full = tt.tt_full(cores)
    for i in range(1, len(shape)):
        lhs = tt.separation(full, i)
        rhs = tt.left_part(cores, i) @ tt.right_part(cores, i + 1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
        assert np.linalg.matrix_rank(lhs) == ranks[i]


def test_ttsvd_order2_is_truncated_svd():
    """For m = 2 Algorithm 1 is the truncated SVD: Eckart-Young error, and the
    same rank-r projection as one built from eigenvectors of X X^T."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((9, 7))
    r = 3
    cores = tt.tt_svd_dense(x, [1, r, 1])
    approx = tt.tt_full(cores)
    sv = np.linalg.svd(x, compute_uv=False)
    assert abs(np.linalg.norm(x - approx) ** 2 - np.sum(sv[r:] ** 2)) < 1e-10
    w, v = np.linalg.eigh(x @ x.T)
    u = v[:, np.argsort(w)[::-1][:r]]
    np.testing.assert_allclose(approx, u @ (u.T @ x), atol=1e-11)


def test_ttsvd_recovers_exact_rank_tensor_and_is_left_orthogonal():
    shape, ranks = [4, 5, 3, 4], [1, 2, 3, 2, 1]
    cores = rand_tt(shape, ranks, 4)
    full = tt.tt_full(cores)
    out = tt.tt_svd_dense(full, ranks)
    np.testing.assert_allclose(tt.tt_full(out), full, rtol=1e-11, atol=1e-11)
    for c in out[:-1]:
        l = c.reshape(-1, c.shape[2])
        np.testing.assert_allclose(l.T @ l, np.eye(c.shape[2]), atol=1e-12)


def test_ttsvd_quasi_optimal_bound():
    """||X - TTSVD_r(X)||^2 <= sum_i sum_{j > r_i} sigma_j(X^{<i>})^2 (Oseledets 2011)."""
    rng = np.random.default_rng(5)
    shape, ranks = [4, 3, 5, 4], [1, 2, 3, 2, 1]
    x = rng.standard_normal(shape)
    out = tt.tt_full(tt.tt_svd_dense(x, ranks))
    err = np.linalg.norm(x - out) ** 2
    bound = 0.0
    for i in range(1, len(shape)):
        sv = np.linalg.svd(tt.separation(x, i), compute_uv=False)
        bound += np.sum(sv[ranks[i]:] ** 2)
    assert err <= bound * (1 + 1e-12)
    assert err > 0


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_tt_round_equals_dense_algorithm1(seed):
    """TT-format rounding reproduces Algorithm 1 run on the dense tensor (compared as tensors)."""
    shape, big, small = [4, 5, 3, 4], [1, 4, 6, 4, 1], [1, 2, 3, 2, 1]
    cores = rand_tt(shape, big, seed)
    ref = tt.tt_full(tt.tt_svd_dense(tt.tt_full(cores), small))
    got = tt.tt_full(tt.tt_round(cores, small))
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_norm_dist_inner_match_dense():
    shape, ranks = [3, 4, 5], [1, 2, 3, 1]
    a = rand_tt(shape, ranks, 9)
    b = [c + 1e-7 * np.random.default_rng(10).standard_normal(c.shape) for c in a]
    fa, fb = tt.tt_full(a), tt.tt_full(b)
    assert abs(tt.tt_inner(a, b) - np.sum(fa * fb)) < 1e-10 * np.sum(fa * fa)
    assert abs(tt.tt_norm(a) - np.linalg.norm(fa)) < 1e-12 * np.linalg.norm(fa)
    d = tt.tt_dist(a, b)
    assert abs(d - np.linalg.norm(fa - fb)) < 1e-6 * d


def test_left_orthogonalize_keeps_tensor():
    shape, ranks = [3, 4, 5, 2], [1, 2, 3, 2, 1]
    a = rand_tt(shape, ranks, 11)
    q, rs = tt.left_orthogonalize(a)
    np.testing.assert_allclose(tt.tt_full(q), tt.tt_full(a), rtol=1e-12, atol=1e-12)
    for c, r in zip(q[:-1], rs):
        l = c.reshape(-1, c.shape[2])
        np.testing.assert_allclose(l.T @ l, np.eye(c.shape[2]), atol=1e-13)
        assert np.all(np.diag(r) >= 0)


def test_oversampling_ratio_matches_qst_experiment():
    """Section 5.3: 10 qubits, TT rank 4, OS = 200 gives a sampling ratio of about 7.6%."""
    with open(os.path.join(GOLDEN, "qst_sampling_ratio.json")) as f:
        g = json.load(f)
    shape = [4] * g["qubits"]
    ranks = [1] + [g["rank"]] * (g["qubits"] - 1) + [1]
    dim = tt.manifold_dim(shape, ranks)
    n_obs = g["os"] * dim
    ratio = n_obs / math.prod(shape)
    assert abs(ratio - g["ratio_about"]) < 0.0005


def test_sampler_draws_distinct_uniform_indices():
    rng = wl.make_rng(0)
    idx = wl.sample_indices([7, 5, 6], 150, rng)
    keys = set(map(tuple, idx.T.tolist()))
    assert len(keys) == 150
    big = wl.sample_indices([4] * 20, 5000, wl.make_rng(1))
    assert len(set(map(tuple, big.T.tolist()))) == 5000
    assert big.min() >= 0 and big.max() <= 3
