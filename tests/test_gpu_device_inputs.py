"""Solves created from device buffers: Omega is checked and summarised on the
device (no copy back to the host), so the result must match a solve created
from host arrays, for every sampled-pass family whose chunk tables need
per-slice counts, and bad observation sets must be refused with the same
statuses as from the host.

Cases: order 3 with the grouped pass (middle-mode counts), order 14 with the
chain pass (index-prefix counts), order 5 with the per-mode passes (counts per
mode).  Bars: iterates equal bit for bit (same grouping, same kernels; to
1e-12 for the per-mode passes, whose segment flushes use atomics), and the
reported relative residual within 1e-12 (||y||^2 is summed in another order
on the device).
"""

import sys

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


def case(name):
    if name == "order3":
        return wl.problem([40, 36, 44], [1, 4, 4, 1], 6000, 61, name=name, init_rel=0.1), {}
    if name == "chain14":
        shape = [4] * 14
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 300_000, 62, name=name, init_rel=0.1), \
            {"pass_kind": "chain"}
    if name == "modes5":
        shape = [9, 7, 8, 6, 9]
        return wl.problem(shape, wl.feasible_ranks(shape, 4), 8000, 63, name=name, init_rel=0.1), \
            {"pass_kind": "modes"}
    raise KeyError(name)


@pytest.mark.parametrize("name", ["order3", "chain14", "modes5"])
def test_device_inputs_match_host_inputs(L, name):
    torch = pytest.importorskip("torch")
    pb, kw = case(name)
    say("case", name, pb.shape, pb.n_obs)
    y = tt.tt_eval(pb.truth, pb.indices)
    runs = []
    for dev in (False, True):
        idx = torch.from_numpy(np.ascontiguousarray(pb.indices)).cuda() if dev else pb.indices
        val = torch.from_numpy(np.ascontiguousarray(y)).cuda() if dev else y
        s = L.Solver(pb.shape, pb.ranks, idx, val, pb.init, step=0.9, stop_rule="none", max_iter=3, **kw)
        try:
            s.iterate(3)
            runs.append((s.cores(), s.report()))
        finally:
            s.close()
    (ch, rh), (cd, rd) = runs
    if kw.get("pass_kind") == "modes":
        # the per-mode passes flush their segment sums with atomics, so two
        # runs agree to rounding only, whatever the inputs' memory
        assert tt.tt_dist(cd, ch) <= 1e-12 * tt.tt_norm(ch)
    else:
        for a, b in zip(ch, cd):
            assert np.array_equal(a, b)
    assert abs(rh["rel_residual"] - rd["rel_residual"]) <= 1e-12 * rh["rel_residual"]


def test_bad_device_inputs_are_refused(L):
    torch = pytest.importorskip("torch")
    pb, _ = case("order3")
    y = tt.tt_eval(pb.truth, pb.indices)

    def create(idx, val):
        return L.Solver(pb.shape, pb.ranks, torch.from_numpy(np.ascontiguousarray(idx)).cuda(),
                        torch.from_numpy(np.ascontiguousarray(val)).cuda(), pb.init,
                        stop_rule="none", max_iter=0)

    bad = pb.indices.copy()
    bad[2, 4321] = pb.shape[2]              # one past the last slice of mode 3
    with pytest.raises(L.PrgdError) as ei:
        create(bad, y)
    assert ei.value.status == L.EINVAL and "mode 2 at sample 4321" in str(ei.value)
    bad = pb.indices.copy()
    bad[0, 17] = -1
    with pytest.raises(L.PrgdError) as ei:
        create(bad, y)
    assert ei.value.status == L.EINVAL and "sample 17" in str(ei.value)
    yv = y.copy()
    yv[999] = np.nan
    with pytest.raises(L.PrgdError) as ei:
        create(pb.indices, yv)
    assert ei.value.status == L.EINVAL and "sample 999" in str(ei.value)
    dup = pb.indices.copy()
    dup[:, 5000] = dup[:, 12]               # sample 5000 repeats sample 12
    with pytest.raises(L.PrgdError) as ei:
        create(dup, y)
    assert ei.value.status == L.EDUPLICATE


def test_device_duplicate_check_with_a_wrapping_linear_index(L):
    # 2^13 per mode over 5 modes: the linear index exceeds 2^64, so equal
    # keys are compared index by index; a shape with no repeat must pass
    torch = pytest.importorskip("torch")
    shape = [8192] * 5
    rng = np.random.default_rng(64)
    N = 20000
    idx = np.stack([rng.integers(0, 8192, N) for _ in range(5)]).astype(np.int32)
    # a second sample whose linear index equals the first one's modulo 2^64
    # would be the interesting collision; random draws make none, and an
    # exact repeat must still be found
    ranks = [1, 2, 2, 2, 2, 1]
    init = [np.asarray(rng.standard_normal((ranks[k], shape[k], ranks[k + 1])) * 0.1) for k in range(5)]
    val = np.ones(N)
    s = L.Solver(shape, ranks, torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda(), init,
                 stop_rule="none", max_iter=0)
    s.close()
    idx[:, 777] = idx[:, 3]
    with pytest.raises(L.PrgdError) as ei:
        L.Solver(shape, ranks, torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda(), init,
                 stop_rule="none", max_iter=0)
    assert ei.value.status == L.EDUPLICATE
