"""Quantum-state-tomography workload (section 5.3) on the GPU: 10 qubits, Pauli
measurement tensor of a random MPS with bond 2 (TT ranks 4), OS = 200
(|Omega| = 80,000, about 7.6% of 4^10).  Every float64 iterate within 1e-10 of
the reference, and both precisions recover the tensor to 1e-6."""

import sys

import numpy as np
import pytest

from oracle import prgd, qst, tt
from paper_2501_13385_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2501_13385_amd import _lib
    _lib.load()
    return _lib


@pytest.fixture(scope="module")
def problem():
    rng = wl.make_rng(0)
    mps = wl.random_mps(10, 2, rng)
    truth = qst.measurement_truth(mps)
    shape, ranks = [4] * 10, tt.ranks_of(truth)
    n_obs = 200 * tt.manifold_dim(shape, ranks)
    idx = wl.sample_indices(shape, n_obs, rng)
    init = wl.perturb_cores(truth, 0.1, rng)
    y = tt.tt_eval(truth, idx)
    return shape, ranks, truth, idx, init, y


def rel_dist(a, b):
    return tt.tt_dist(a, b) / tt.tt_norm(b)


@pytest.mark.parametrize("rule,iters", [("theory", 4), ("adaptive", 3)])
def test_qst_iterates_match_reference(L, problem, rule, iters):
    shape, ranks, truth, idx, init, y = problem
    print("qst", rule, idx.shape, flush=True)
    pol = prgd.Policy(step_rule=rule, c=1.0)
    s = L.Solver(shape, ranks, idx, y, init, step=1.0, step_policy=rule, stop_rule="none", max_iter=iters)
    ref = [c.copy() for c in init]
    try:
        for it in range(iters):
            s.iterate(1)
            got = s.cores()
            ref, _ = prgd.prgd_step(ref, idx, y, pol, ranks)
            d = rel_dist(got, ref)
            assert d <= 1e-10, (it, d)
    finally:
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_qst_recovery_to_1e6(L, problem, precision):
    shape, ranks, truth, idx, init, y = problem
    v = y if precision == "fp64" else y.astype(np.float32)
    s = L.Solver(shape, ranks, idx, v, init, truth_cores=truth, precision=precision, step=1.0,
                 stop_rule="error", tol=1e-6, max_iter=200)
    try:
        rep = s.run()
        got = s.cores()
    finally:
        s.close()
    print("qst", precision, rep, flush=True)
    assert rep["status"] == 0
    assert rel_dist(got, truth) <= 1e-6
