"""Pins of the reference's sketched spectral initialisation
(``oracle.prgd.spectral_init_sketch``): exact recovery of an exact-rank
tensor observed in full, agreement with the dense Algorithm 1 when the sketch
is an isometry (order 2), agreement with a brute-force dense sketch (every
index tuple enumerated) at partial observation, and left-orthonormal cores."""

import itertools

import numpy as np
import pytest

from oracle import prgd, tt
from paper_2501_13385_amd import workloads as wl


def rel(a, b):
    return tt.tt_dist(a, b) / tt.tt_norm(b)


@pytest.mark.parametrize("shape,ranks", [([6, 7, 5], [1, 3, 2, 1]), ([4, 5, 3, 4], [1, 2, 3, 2, 1]), ([9, 8], [1, 3, 1])])
def test_exact_rank_tensor_observed_in_full_is_recovered(shape, ranks):
    rng = wl.make_rng(11)
    truth = wl.gaussian_cores(shape, ranks, rng)
    full = np.array(np.unravel_index(np.arange(int(np.prod(shape))), shape), dtype=np.int32)
    y = tt.tt_eval(truth, full)
    g = wl.sketch_gaussians(shape, max(ranks) + 2, rng)
    got = prgd.spectral_init_sketch(full, y, shape, ranks, g)
    assert rel(got, truth) <= 1e-12


def test_isometric_sketch_equals_dense_tt_svd_order2():
    # one later mode: Psi = Gamma with orthonormal rows, so Y Y^T = A A^T
    rng = wl.make_rng(12)
    shape, ranks, s = [7, 5], [1, 2, 1], 6
    truth = wl.gaussian_cores(shape, ranks, rng)
    idx = wl.sample_indices(shape, 20, rng)
    y = tt.tt_eval(truth, idx) + 0.05 * rng.standard_normal(20)
    q, _ = np.linalg.qr(rng.standard_normal((s, s)))
    got = prgd.spectral_init_sketch(idx, y, shape, ranks, [q[: shape[1], :]])
    ref = prgd.spectral_init_dense(idx, y, shape, ranks)
    assert rel(got, ref) <= 1e-12


def brute_force_sketch_init(idx, y, shape, ranks, gauss):
    """The same algorithm on the dense zero-filled tensor, with every test
    matrix Psi_i materialised by enumerating all later index tuples."""
    m = len(shape)
    z = np.zeros(shape)
    z[tuple(idx)] = y
    z /= idx.shape[1] / np.prod(shape)
    left = np.ones((1, 1))
    cores, g = [], 0
    for i in range(m - 1):
        later = list(range(i + 1, m))
        gam = [np.asarray(gauss[g + t]) for t in range(len(later))]
        g += len(later)
        s = gam[0].shape[1]
        tuples = list(itertools.product(*[range(shape[k]) for k in later]))
        psi = np.ones((len(tuples), s))
        for row, tup in enumerate(tuples):
            for t, xk in enumerate(tup):
                psi[row] *= gam[t][xk]
        zi = z.reshape(left.shape[0], shape[i], -1)
        mat = np.einsum("pj,pxr->jxr", left, zi).reshape(left.shape[1] * shape[i], -1)
        u, _, _ = np.linalg.svd(mat @ psi, full_matrices=False)
        core = u[:, : ranks[i + 1]].reshape(left.shape[1], shape[i], ranks[i + 1])
        cores.append(core)
        left = (left @ core.reshape(core.shape[0], -1)).reshape(-1, ranks[i + 1])
    last = left.T @ z.reshape(left.shape[0], -1)
    cores.append(last.reshape(last.shape[0], shape[-1], 1))
    return cores


@pytest.mark.parametrize("shape,ranks,n_obs", [([5, 6, 4], [1, 3, 2, 1], 50), ([4, 3, 5, 4], [1, 2, 3, 2, 1], 120)])
def test_agrees_with_brute_force_dense_sketch(shape, ranks, n_obs):
    rng = wl.make_rng(13)
    truth = wl.gaussian_cores(shape, ranks, rng)
    idx = wl.sample_indices(shape, n_obs, rng)
    y = tt.tt_eval(truth, idx) + 0.05 * rng.standard_normal(n_obs)
    g = wl.sketch_gaussians(shape, max(ranks) + 3, rng)
    got = prgd.spectral_init_sketch(idx, y, shape, ranks, g)
    ref = brute_force_sketch_init(idx, y, shape, ranks, g)
    assert rel(got, ref) <= 1e-11


def test_cores_are_left_orthonormal():
    rng = wl.make_rng(14)
    shape, ranks = [8, 6, 7, 5], [1, 3, 4, 2, 1]
    truth = wl.gaussian_cores(shape, ranks, rng)
    idx = wl.sample_indices(shape, 400, rng)
    y = tt.tt_eval(truth, idx)
    got = prgd.spectral_init_sketch(idx, y, shape, ranks, wl.sketch_gaussians(shape, 6, rng))
    for c in got[:-1]:
        u = c.reshape(-1, c.shape[2])
        assert np.abs(u.T @ u - np.eye(u.shape[1])).max() <= 1e-13


def test_too_few_samples_is_reported():
    rng = wl.make_rng(15)
    shape, ranks = [6, 6, 6], [1, 3, 3, 1]
    idx = wl.sample_indices(shape, 2, rng)       # sketch of rank <= 2 < r_1
    with pytest.raises(ValueError):
        prgd.spectral_init_sketch(idx, np.ones(2), shape, ranks, wl.sketch_gaussians(shape, 5, rng))


def test_small_but_resolvable_singular_values_are_kept():
    """Algorithm 1 keeps the top r singular vectors whatever their scale; only a
    rank that float64 cannot resolve is refused.  A fully observed tensor whose
    r-th sketch singular value is about 1e-10 of the largest (far below the
    square root of machine precision, far above its rounding level) is still
    reproduced."""
    from oracle import tt as _tt
    shape, ranks = [6, 5, 7], [1, 2, 2, 1]
    rng = wl.make_rng(16)
    big = wl.gaussian_cores(shape, [1, 1, 1, 1], rng)
    small = wl.gaussian_cores(shape, [1, 1, 1, 1], rng)
    small[0] = small[0] * 1e-10
    truth = _tt.tt_add(big, small)                 # TT rank (1, 2, 2, 1), sigma_2 / sigma_1 ~ 1e-10
    full = np.array(np.unravel_index(np.arange(int(np.prod(shape))), shape)).astype(np.int32)
    y = _tt.tt_eval(truth, full)
    got = prgd.spectral_init_sketch(full, y, shape, ranks, wl.sketch_gaussians(shape, 5, rng))
    assert rel(got, truth) <= 1e-12
    # the small component itself is recovered, not only the dominant one
    diff = _tt.tt_add(got, big, -1.0)
    assert _tt.tt_dist(diff, small) <= 1e-4 * _tt.tt_norm(small)
