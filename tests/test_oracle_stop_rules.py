"""Pins for the stopping quantities of the reference loop (``oracle.prgd.prgd``):
relative residual, relative change and relative error recomputed from the
dense tensors of the kept iterates (section 5.1 rules: the change
||T_{l+1} - T_l||_F / max(1, ||T_l||_F), the error ||T_{l+1} - T*||_F / ||T*||_F,
and the residual ||P_Omega T_l - y|| / ||y||).  Two scales are used so that both
branches of max(1, ||T_l||) are exercised, and starts far from the truth so
that ||T_l|| and ||T_{l+1}|| differ by much more than the tolerance (a change
normalised by the wrong iterate fails)."""

import numpy as np
import pytest

from oracle import prgd, tt
from paper_2501_13385_amd import workloads as wl


def _case(scale, seed):
    shape, ranks = [4, 5, 3], [1, 2, 2, 1]
    rng = wl.make_rng(seed)
    truth = wl.gaussian_cores(shape, ranks, rng)
    truth[0] = truth[0] * scale
    init = wl.perturb_cores(truth, 0.6, rng)
    idx = wl.sample_indices(shape, 45, rng)
    y = tt.tt_eval(truth, idx)
    return shape, ranks, truth, init, idx, y


@pytest.mark.parametrize("scale,seed", [(3.0, 40), (0.02, 41)])
def test_change_error_residual_match_dense_tensors(scale, seed):
    shape, ranks, truth, init, idx, y = _case(scale, seed)
    pol = prgd.Policy(step_rule="theory", c=0.7, stop_rule="change", tol=0.0, max_iter=6)
    res = prgd.prgd(init, idx, y, pol, truth=truth, keep_iterates=True)
    dense = [tt.tt_full(c) for c in res.iterates]
    dstar = tt.tt_full(truth)
    norms = [np.linalg.norm(d) for d in dense]
    # the two branches of max(1, ||T_l||) and distinct consecutive norms
    assert (min(norms) > 1.0) if scale > 1 else (max(norms) < 1.0)
    assert max(abs(norms[i + 1] - norms[i]) / norms[i] for i in range(len(norms) - 1)) > 1e-3
    assert len(res.history) == 6
    for h in res.history:
        l = h["iter"]
        want_change = np.linalg.norm(dense[l + 1] - dense[l]) / max(1.0, np.linalg.norm(dense[l]))
        want_err = np.linalg.norm(dense[l + 1] - dstar) / np.linalg.norm(dstar)
        want_res = np.linalg.norm(dense[l][tuple(idx)] - y) / np.linalg.norm(y)
        assert h["rel_change"] == pytest.approx(want_change, rel=1e-10)
        assert h["rel_err"] == pytest.approx(want_err, rel=1e-10)
        assert h["rel_res"] == pytest.approx(want_res, rel=1e-10)


def test_change_rule_stops_at_first_iterate_below_tolerance():
    shape, ranks, truth, init, idx, y = _case(3.0, 42)
    free = prgd.prgd(init, idx, y, prgd.Policy(c=0.7, stop_rule="change", tol=0.0, max_iter=12), keep_iterates=True)
    ch = [h["rel_change"] for h in free.history]
    tol = float(np.median(ch))
    first = next(i for i, c in enumerate(ch) if c <= tol)
    res = prgd.prgd(init, idx, y, prgd.Policy(c=0.7, stop_rule="change", tol=tol, max_iter=12))
    assert res.status == "converged"
    assert res.iterations == first + 1
    assert all(np.array_equal(a, b) for a, b in zip(res.cores, free.iterates[first + 1]))


def test_error_rule_stops_at_first_iterate_below_tolerance():
    shape, ranks, truth, init, idx, y = _case(3.0, 43)
    free = prgd.prgd(init, idx, y, prgd.Policy(c=0.7, stop_rule="change", tol=0.0, max_iter=12), truth=truth,
                     keep_iterates=True)
    errs = [np.linalg.norm(tt.tt_full(c) - tt.tt_full(truth)) / np.linalg.norm(tt.tt_full(truth))
            for c in free.iterates[1:]]
    tol = float(np.median(errs))
    first = next(i for i, e in enumerate(errs) if e <= tol)
    res = prgd.prgd(init, idx, y, prgd.Policy(c=0.7, stop_rule="error", tol=tol, max_iter=12), truth=truth)
    assert res.status == "converged"
    assert res.iterations == first + 1
