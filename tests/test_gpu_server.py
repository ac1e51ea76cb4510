"""Request server (continuous batching): every result equals the same problem
solved alone, admission respects the memory budget, solves overlap on the
device, and invalid or oversized requests are refused.

Bars: float64 requests, final iterate within 1e-10 relative of the solve
alone (the per-iteration float64 parity bar) and the same iteration count;
mixed-precision requests, final relative recovery error within 1e-5 of the
solve alone.
"""

import sys
import time

import numpy as np
import pytest

from oracle import tt
from paper_2501_13385_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2501_13385_amd import _lib
    _lib.load()
    return _lib


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_dist(a, b):
    return tt.tt_dist(a, b) / tt.tt_norm(b)


def observed(pb):
    return tt.tt_eval(pb.truth, pb.indices) + pb.noise_std * pb.noise


def mix():
    """Problems of several orders, ranks, sizes and both precisions; the two order-6 ones share a batch group."""
    out = []
    out.append((wl.named("c1"), dict(step=1.001, stop_rule="residual", tol=1e-10, max_iter=500)))
    out.append((wl.named("c2_small"), dict(step=0.8, stop_rule="change", tol=1e-6, max_iter=200)))
    out.append((wl.problem([30, 50, 40], [1, 4, 4, 1], 5000, 11, name="o3b", init_rel=0.1),
                dict(step=0.8, stop_rule="residual", tol=1e-9, max_iter=300)))
    out.append((wl.problem([7, 11, 5, 9], [1, 3, 5, 2, 1], 1500, 3, name="ragged", init_rel=0.1),
                dict(step=0.8, stop_rule="residual", tol=1e-9, max_iter=300)))
    out.append((wl.problem([37, 29], [1, 3, 1], 400, 5, name="order2", init_rel=0.2),
                dict(step=0.8, stop_rule="residual", tol=1e-9, max_iter=300)))
    shape = [3, 4, 3, 5, 3, 4]
    out.append((wl.problem(shape, wl.feasible_ranks(shape, 4), 1200, 6, name="order6", init_rel=0.1),
                dict(step=0.8, stop_rule="none", max_iter=15)))
    out.append((wl.named("c2_small", seed=4), dict(step=0.8, stop_rule="change", tol=1e-6, max_iter=200,
                                                   precision="mixed")))
    # a second order-6 problem of the same ranks: the two share a launch of the
    # one-workgroup dense kernels (mode sizes <= 8, padded rank 4)
    out.append((wl.problem(shape, wl.feasible_ranks(shape, 4), 1300, 16, name="order6b", init_rel=0.1),
                dict(step=0.8, stop_rule="none", max_iter=15)))
    return out


def alone(L, pb, kw):
    y = observed(pb)
    if kw.get("precision") == "mixed":
        y = y.astype(np.float32)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, truth_cores=pb.truth, **kw)
    try:
        rep = s.run()
        cores = s.cores()
    finally:
        s.close()
    return rep, cores


def submit(L, sv, pb, kw):
    y = observed(pb)
    if kw.get("precision") == "mixed":
        y = y.astype(np.float32)
    return sv.submit(pb.shape, pb.ranks, pb.indices, y, pb.init, truth_cores=pb.truth, **kw)


def check_same(pb, kw, ref, got):
    (rrep, rcores), (st, info, cores) = ref, got
    assert st in (L_OK, L_NOT_CONVERGED), st
    if kw.get("precision") == "mixed":
        assert abs(rel_dist(cores, pb.truth) - rel_dist(rcores, pb.truth)) <= 1e-5
    else:
        assert info["iterations"] == rrep["iterations"], (pb.name, info["iterations"], rrep["iterations"])
        d = rel_dist(cores, rcores)
        say(pb.name, "iterations", info["iterations"], "difference to the solve alone", d)
        assert d <= 1e-10, (pb.name, d)
    for core in cores[:-1]:
        lm = core.reshape(-1, core.shape[2])
        np.testing.assert_allclose(lm.T @ lm, np.eye(core.shape[2]), atol=1e-10)


L_OK, L_NOT_CONVERGED = 0, 1


def test_mix_results_equal_solves_alone(L):
    cases = mix()
    refs = [alone(L, pb, kw) for pb, kw in cases]
    with L.Server(max_slots=64, iters_per_tick=3) as sv:
        tickets = [submit(L, sv, pb, kw) for pb, kw in cases]
        got = [sv.result(t, 120.0) for t in tickets]
    for (pb, kw), ref, g in zip(cases, refs, got):
        assert g is not None, pb.name
        check_same(pb, kw, ref, g)


def test_staggered_arrivals_overlap_and_match(L):
    cases = mix()[:5]
    refs = [alone(L, pb, kw) for pb, kw in cases]
    with L.Server(max_slots=64, iters_per_tick=1) as sv:
        tickets = []
        for pb, kw in cases:
            tickets.append(submit(L, sv, pb, kw))
            time.sleep(0.002)
        got = [sv.result(t, 120.0) for t in tickets]
    infos = [g[1] for g in got]
    # some solve was admitted while another was still running on the device
    overlap = any(a["admit_s"] < b["finish_s"] and b["admit_s"] < a["finish_s"]
                  for i, a in enumerate(infos) for b in infos[i + 1:])
    say("admission/finish", [(round(i["admit_s"], 4), round(i["finish_s"], 4)) for i in infos])
    assert overlap
    for (pb, kw), ref, g in zip(cases, refs, got):
        check_same(pb, kw, ref, g)


def test_budget_admits_one_at_a_time_when_only_one_fits(L):
    cases = mix()[:4]
    refs = [alone(L, pb, kw) for pb, kw in cases]
    # a budget just above the largest request: never two resident at once
    big = 0
    with L.Server(max_slots=8) as sv0:
        for pb, kw in cases:
            t = submit(L, sv0, pb, kw)
            big = max(big, sv0.result(t, 120.0)[1]["footprint_bytes"])
    with L.Server(hbm_budget_bytes=big + 1024, max_slots=8) as sv:
        tickets = [submit(L, sv, pb, kw) for pb, kw in cases]
        got = [sv.result(t, 120.0) for t in tickets]
    spans = sorted((g[1]["admit_s"], g[1]["finish_s"]) for g in got)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0, spans
    for (pb, kw), ref, g in zip(cases, refs, got):
        check_same(pb, kw, ref, g)


def test_oversize_and_invalid_requests_are_refused(L):
    pb = wl.named("c1")
    y = observed(pb)
    with L.Server(hbm_budget_bytes=1 << 16, max_slots=4) as sv:
        with pytest.raises(L.PrgdError) as e:
            sv.submit(pb.shape, pb.ranks, pb.indices, y, pb.init)
        assert e.value.status == L.ENOMEM
    with L.Server(max_slots=4) as sv:
        idx = pb.indices.copy()
        idx[:, 1] = idx[:, 0]
        with pytest.raises(L.PrgdError) as e:
            sv.submit(pb.shape, pb.ranks, idx, y, pb.init)
        assert e.value.status == L.EDUPLICATE
        t = sv.submit(pb.shape, pb.ranks, pb.indices, y, pb.init, step=1.001, tol=1e-10)
        assert sv.wait(t, 60.0)
        st, info, cores = sv.poll(t)
        assert st == 0 and info["rel_residual"] <= 1e-10
        with pytest.raises(L.PrgdError):
            L.prgd_server_poll(sv.h, t)          # released
