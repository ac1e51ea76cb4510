"""Pins for the reference PRGD (oracle/prgd.py): brute force, finite differences,
defining properties, invariances and recovery."""

import itertools
import math

import numpy as np
import pytest

from oracle import prgd, tt
from paper_2501_13385_amd import workloads as wl


def rand_tt(shape, ranks, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal((ranks[k], shape[k], ranks[k + 1])) for k in range(len(shape))]


def tiny_problem(seed=0, shape=(3, 4, 5), ranks=(1, 2, 2, 1), frac=0.6):
    shape, ranks = list(shape), list(ranks)
    rng = np.random.default_rng(seed)
    truth = rand_tt(shape, ranks, seed + 100)
    cores = [c + 0.3 * rng.standard_normal(c.shape) for c in truth]
    cores, _ = tt.left_orthogonalize(cores)
    total = int(np.prod(shape))
    n_obs = int(frac * total)
    lin = rng.choice(total, n_obs, replace=False)
    idx = np.array(np.unravel_index(lin, shape))
    y = tt.tt_eval(truth, idx)
    return shape, ranks, truth, cores, idx, y


def dense_gradient(shape, idx, r):
    g = np.zeros(shape)
    g[tuple(idx)] = r
    return g


def jacobian(cores):
    """Columns d vec(T) / d T_i(a,x,b): the tensor with core i replaced by a unit core."""
    cols = []
    for i, c in enumerate(cores):
        for pos in itertools.product(*[range(s) for s in c.shape]):
            e = np.zeros_like(c)
            e[pos] = 1.0
            cc = list(cores)
            cc[i] = e
            cols.append(tt.tt_full(cc).ravel())
    return np.stack(cols, axis=1)


def test_slice_norms_are_row_norms_of_dense_unfoldings():
    shape, ranks, truth, cores, idx, y = tiny_problem(1)
    r = prgd.residual(cores, idx, y)
    s = prgd.slice_norms(idx, r, shape)
    gd = dense_gradient(shape, idx, r)
    for i in range(len(shape)):
        m = tt.mode_unfolding(gd, i)
        np.testing.assert_allclose(s[i], np.sum(m * m, axis=1), rtol=1e-13, atol=1e-15)
    assert prgd.eps_vee(s) == pytest.approx(max(np.max(np.sum(tt.mode_unfolding(gd, i) ** 2, axis=1))
                                              for i in range(3)))


def test_core_gradient_matches_central_differences():
    shape, ranks, truth, cores, idx, y = tiny_problem(2)

    def f(cs):
        rr = tt.tt_eval(cs, idx) - y
        return 0.5 * float(rr @ rr)

    grads = prgd.core_gradient(cores, idx, prgd.residual(cores, idx, y))
    h = 1e-6
    for i, c in enumerate(cores):
        for pos in itertools.product(*[range(s) for s in c.shape]):
            cp = [x.copy() for x in cores]
            cm = [x.copy() for x in cores]
            cp[i][pos] += h
            cm[i][pos] -= h
            fd = (f(cp) - f(cm)) / (2 * h)
            assert abs(fd - grads[i][pos]) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("seed,shape,ranks", [
    (3, (3, 4, 5), (1, 2, 2, 1)),
    (4, (3, 3, 2, 4), (1, 2, 3, 2, 1)),
    (5, (4, 5), (1, 2, 1)),
])
def test_direction_equals_brute_force_weighted_projection(seed, shape, ranks):
    """xi = P~_T W^{-1} G equals the W-orthogonal projection onto range(J) of W^{-1} G,
    with J the Jacobian of the TT map and W = diag(prod_k g_k(x_k)^{1/(2m)}) built from
    dense mode unfoldings (section 3.2: metric, Riemannian gradient)."""
    shape, ranks, truth, cores, idx, y = tiny_problem(seed, shape, ranks)
    m = len(shape)
    r = prgd.residual(cores, idx, y)
    gd = dense_gradient(shape, idx, r)
    gdiag = []
    for i in range(m):
        u = tt.mode_unfolding(gd, i)
        gdiag.append(np.sum(u * u, axis=1))
    eps = max(x.max() for x in gdiag)
    gdiag = [eps + x for x in gdiag]
    w = np.ones(shape)
    for i in range(m):
        sh = [1] * m
        sh[i] = shape[i]
        w = w * (gdiag[i] ** (1.0 / (2 * m))).reshape(sh)
    target = (gd / w).ravel()
    jac = jacobian(cores)
    sw = np.sqrt(w.ravel())
    theta, *_ = np.linalg.lstsq(sw[:, None] * jac, sw * target, rcond=None)
    ref = jac @ theta

    d = prgd.tangent_direction(cores, idx, r)
    got = tt.tt_full(prgd.tangent_tt(d.base, d.comps)).ravel()
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    # defining property of the Riemannian gradient: <xi, eta>_W = <G, eta> for tangent eta
    eta = jac @ np.random.default_rng(seed).standard_normal(jac.shape[1])
    assert abs(np.sum(w.ravel() * got * eta) - np.sum(gd.ravel() * eta)) <= 1e-10 * np.linalg.norm(gd) * np.linalg.norm(eta)


def test_gauge_lemma1_lemma2():
    """Gauge L(T^_i)^T L(A^_i) = 0 (section 3.3), Lemma 1 (weighted orthogonality of
    the new left parts) and Lemma 2 (W-orthogonality of the components)."""
    shape, ranks, truth, cores, idx, y = tiny_problem(6, (3, 4, 3, 4), (1, 2, 3, 2, 1))
    m = len(shape)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r)
    for i in range(m - 1):
        lt = d.hat_base[i].reshape(-1, d.hat_base[i].shape[2])
        la = d.hat_comps[i].reshape(-1, d.hat_comps[i].shape[2])
        assert np.abs(lt.T @ la).max() <= 1e-12 * max(1.0, np.abs(la).max())
    # Lemma 1
    for i in range(1, m):
        left = tt.left_part(d.base, i)
        wd = np.ones(1)
        for k in range(i):
            wd = np.kron(wd, d.g[k] ** (1.0 / (2 * m)))
        np.testing.assert_allclose(left.T @ (wd[:, None] * left), np.eye(left.shape[1]), atol=1e-12)
    # Lemma 2
    w = np.ones(shape)
    for i in range(m):
        sh = [1] * m
        sh[i] = shape[i]
        w = w * (d.g[i] ** (1.0 / (2 * m))).reshape(sh)
    terms = []
    for i in range(m):
        cc = list(d.base)
        cc[i] = d.comps[i]
        terms.append(tt.tt_full(cc))
    for i in range(m):
        for j in range(i + 1, m):
            ip = np.sum(w * terms[i] * terms[j])
            assert abs(ip) <= 1e-11 * np.linalg.norm(terms[i]) * np.linalg.norm(terms[j])


def test_uniform_weights_give_euclidean_projection():
    """With equal metric weights PRGD's projection is the Euclidean tangent projection
    (the RGD special case): compare with the unweighted brute-force projector."""
    shape, ranks, truth, cores, idx, y = tiny_problem(7)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r, eps=1e30)     # g ~ eps, s negligible
    got = tt.tt_full(prgd.tangent_tt(d.base, d.comps)).ravel()
    jac = jacobian(cores)
    gd = dense_gradient(shape, idx, r).ravel()
    theta, *_ = np.linalg.lstsq(jac, gd, rcond=None)
    ref = (jac @ theta) / math.sqrt(1e30)       # W^{-1} = eps^{-1/2} I
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_adaptive_step_minimises_linearised_objective():
    """eq. "PRGD stepsize": alpha* = argmin_a f(T - a xi) over the tangent line."""
    shape, ranks, truth, cores, idx, y = tiny_problem(8)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r)
    a = prgd.step_adaptive(d, idx)
    xi = tt.tt_full(prgd.tangent_tt(d.base, d.comps))
    full = tt.tt_full(cores)

    def f(al):
        v = (full - al * xi)[tuple(idx)] - y
        return 0.5 * float(v @ v)

    # f is quadratic in the step: its minimiser from three samples
    f0, f1, f2 = f(0.0), f(1.0), f(2.0)
    amin = (3 * f0 - 4 * f1 + f2) / (2 * (f0 - 2 * f1 + f2))
    assert abs(a - amin) <= 1e-9 * abs(amin)


def test_step_update_and_retraction_dense():
    """One iteration equals Algorithm 1 applied to the dense T_l - alpha xi, and the
    block TT of W_l equals that dense tensor."""
    shape, ranks, truth, cores, idx, y = tiny_problem(9, (3, 4, 3, 4), (1, 2, 3, 2, 1))
    pol = prgd.Policy(step_rule="theory", c=0.8)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r)
    p = len(y) / np.prod(shape)
    alpha = 0.8 * math.sqrt(d.eps) / p
    wdense = tt.tt_full(cores) - alpha * tt.tt_full(prgd.tangent_tt(d.base, d.comps))
    wblock = tt.tt_full(prgd.tangent_tt(d.base, d.comps, -alpha, add_base=True))
    np.testing.assert_allclose(wblock, wdense, atol=1e-12 * np.abs(wdense).max())
    new, info = prgd.prgd_step(cores, idx, y, pol, ranks)
    assert info["alpha"] == pytest.approx(alpha, rel=1e-14)
    ref = tt.tt_full(tt.tt_svd_dense(wdense, ranks))
    np.testing.assert_allclose(tt.tt_full(new), ref, atol=1e-10 * np.abs(ref).max())


def _run(cores, idx, y, iters=5, c=0.8):
    pol = prgd.Policy(step_rule="theory", c=c, stop_rule="residual", tol=0.0, max_iter=iters)
    return prgd.prgd(cores, idx, y, pol)


def test_invariance_gauge_order_and_scale():
    shape, ranks, truth, cores, idx, y = tiny_problem(10, (4, 3, 4, 3), (1, 2, 3, 2, 1), frac=0.7)
    base = tt.tt_full(_run(cores, idx, y).cores)
    # random gauge at every bond leaves the tensor and the iterates unchanged
    rng = np.random.default_rng(0)
    g = [c.copy() for c in cores]
    for k in range(len(g) - 1):
        q = rng.standard_normal((ranks[k + 1], ranks[k + 1])) + 3 * np.eye(ranks[k + 1])
        g[k] = np.einsum("axb,bc->axc", g[k], q)
        g[k + 1] = np.einsum("cb,bxd->cxd", np.linalg.inv(q), g[k + 1])
    np.testing.assert_allclose(tt.tt_full(_run(g, idx, y).cores), base, atol=1e-10 * np.abs(base).max())
    # order of the samples does not matter
    perm = rng.permutation(idx.shape[1])
    np.testing.assert_allclose(tt.tt_full(_run(cores, idx[:, perm], y[perm]).cores), base,
                               atol=1e-10 * np.abs(base).max())
    # scaling T* and T_0 by c scales every iterate by c (theory step)
    c = -3.0
    sc = [x.copy() for x in cores]
    sc[0] = c * sc[0]
    np.testing.assert_allclose(tt.tt_full(_run(sc, idx, c * y).cores), c * base, atol=1e-9 * np.abs(base).max())


def test_noiseless_c1_recovers_to_1e10():
    pb = wl.named("c1")
    y = tt.tt_eval(pb.truth, pb.indices)
    pol = prgd.Policy(step_rule="theory", c=1.001, stop_rule="residual", tol=1e-10, max_iter=500)
    res = prgd.prgd(pb.init, pb.indices, y, pol, truth=pb.truth)
    assert res.status == "converged"
    assert res.iterations < 500
    assert tt.tt_dist(res.cores, pb.truth) / tt.tt_norm(pb.truth) < 1e-9
    rel = [h["rel_err"] for h in res.history if "rel_err" in h]
    rate = (rel[-1] / rel[len(rel) // 2]) ** (1.0 / (len(rel) - 1 - len(rel) // 2))
    assert rate < 0.9


def test_spectral_init_is_rank_r_and_closer_than_zero():
    shape, ranks, truth, cores, idx, y = tiny_problem(11, (5, 6, 5), (1, 2, 2, 1), frac=0.7)
    t0 = prgd.spectral_init_dense(idx, y, shape, ranks)
    assert tt.ranks_of(t0) == ranks
    assert tt.tt_dist(t0, truth) < tt.tt_norm(truth)


def test_euclidean_metric_is_the_euclidean_tangent_projection():
    """metric="euclidean" (RGD, section 3.1): the direction is the orthogonal projection
    of the dense gradient onto the tangent space, computed here by least squares on the
    tangent-space Jacobian (no weights, no eps)."""
    shape, ranks, truth, cores, idx, y = tiny_problem(11, (3, 4, 3), (1, 2, 2, 1))
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r, metric="euclidean")
    got = tt.tt_full(prgd.tangent_tt(d.base, d.comps)).ravel()
    jac = jacobian(cores)
    gd = dense_gradient(shape, idx, r).ravel()
    theta, *_ = np.linalg.lstsq(jac, gd, rcond=None)
    ref = jac @ theta
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_rgd_adaptive_step_minimises_linearised_objective():
    """Section 3.1: alpha = ||P_T G||^2 / ||P_Omega P_T G||^2 minimises f(T - a P_T G)."""
    shape, ranks, truth, cores, idx, y = tiny_problem(12)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r, metric="euclidean")
    a = prgd.step_adaptive(d, idx)
    xi = tt.tt_full(prgd.tangent_tt(d.base, d.comps))
    full = tt.tt_full(cores)

    def f(al):
        v = (full - al * xi)[tuple(idx)] - y
        return 0.5 * float(v @ v)

    f0, f1, f2 = f(0.0), f(1.0), f(2.0)
    amin = (3 * f0 - 4 * f1 + f2) / (2 * (f0 - 2 * f1 + f2))
    assert abs(a - amin) <= 1e-9 * abs(amin)
    pg = float(np.sum(xi * xi))
    pog = float(np.sum(xi[tuple(idx)] ** 2))
    assert abs(a - pg / pog) <= 1e-11 * a


@pytest.mark.parametrize("metric,rule,c", [("euclidean", "adaptive", 1.0), ("euclidean", "theory", 0.8),
                                           ("data", "adaptive", 1.0)])
def test_noiseless_c1_recovery_other_policies(metric, rule, c):
    """RGD (adaptive and constant step) and PRGD with the adaptive step also recover the
    noiseless order-4 problem to 1e-10."""
    pb = wl.named("c1")
    y = tt.tt_eval(pb.truth, pb.indices)
    pol = prgd.Policy(step_rule=rule, c=c, metric=metric, stop_rule="residual", tol=1e-10, max_iter=500)
    res = prgd.prgd(pb.init, pb.indices, y, pol, truth=pb.truth)
    assert res.status == "converged"
    assert tt.tt_dist(res.cores, pb.truth) / tt.tt_norm(pb.truth) <= 1e-9


def test_direction_is_the_riemannian_gradient_under_the_metric():
    """Section 3.2.2: xi = P~_T W^{-1} G is the gradient of f in the metric W restricted to
    the tangent space, so <xi, eta>_W = <G, eta> for every tangent eta (dense check with
    W = x_i G_i^{1/(2m)} applied entrywise, random tangent vectors)."""
    shape, ranks, truth, cores, idx, y = tiny_problem(13, (3, 4, 3), (1, 2, 2, 1))
    m = len(shape)
    r = prgd.residual(cores, idx, y)
    d = prgd.tangent_direction(cores, idx, r)
    xi = tt.tt_full(prgd.tangent_tt(d.base, d.comps))
    w = np.ones(shape)
    for i in range(m):
        sh = [1] * m
        sh[i] = shape[i]
        w = w * (d.g[i] ** (1.0 / (2 * m))).reshape(sh)
    g = dense_gradient(shape, idx, r)
    jac = jacobian(cores)
    rng = np.random.default_rng(3)
    for _ in range(3):
        eta = (jac @ rng.standard_normal(jac.shape[1])).reshape(shape)     # a tangent vector
        lhs = float(np.sum(w * xi * eta))
        rhs = float(np.sum(g * eta))
        assert abs(lhs - rhs) <= 1e-11 * (abs(rhs) + np.linalg.norm(g) * np.linalg.norm(eta))


def test_component_weighted_representation():
    """Proposition 1: W^{1/2} T has the TT cores T_i x_2 G_i^{1/(4m)}."""
    shape, ranks, truth, cores, idx, y = tiny_problem(14, (3, 4, 5), (1, 2, 2, 1))
    m = len(shape)
    rng = np.random.default_rng(4)
    g = [1.0 + rng.random(n) for n in shape]
    scaled = [prgd.scale_mode(cores[k], g[k] ** (1.0 / (4 * m))) for k in range(m)]
    w = np.ones(shape)
    for i in range(m):
        sh = [1] * m
        sh[i] = shape[i]
        w = w * (g[i] ** (1.0 / (4 * m))).reshape(sh)
    np.testing.assert_allclose(tt.tt_full(scaled), w * tt.tt_full(cores), rtol=1e-13, atol=1e-15)
