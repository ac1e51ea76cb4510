"""GPU parity of the order-3 sampled pass for low ranks (padded rank <= 4),
where every chunk of the samples is one wave with a private LDS table of
boundary-core gradients and slice sums, through the C ABI.

The cases cover chunks inside one long middle-mode segment (the slots of
several chunks summed for one segment), chunks spanning many short segments
(segments wholly inside a chunk written directly), middle-mode slices with no
sample, a single partial batch, ragged ranks padded to 2 and 4, and a
million-sample shape with many chunks.

Bars: float64 gradient entries within 1e-12 of the largest entry of their
core (sums in another order), slice sums to 1e-12 relative, and a second pass
identical bit for bit (no two waves add into the same word, so the order of
every sum is fixed); mixed precision within the float32 bound
4e-6 * order * (sum over the samples of |R_j l r|).
"""

import sys

import numpy as np
import pytest

from oracle import prgd, tt
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
    if name == "long_segments":     # 3 middle slices, 60,000 samples: each segment spans many chunks
        return wl.problem([200, 3, 150], [1, 2, 2, 1], 60_000, 41, name=name, init_rel=0.1)
    if name == "short_segments":    # 900 middle slices, 5,000 samples: chunks span many segments
        return wl.problem([30, 900, 25], [1, 2, 2, 1], 5_000, 42, name=name, init_rel=0.1)
    if name == "ragged_r3":         # ranks 3 padded to 4, uneven modes
        return wl.problem([37, 61, 23], [1, 3, 3, 1], 40_000, 43, name=name, init_rel=0.1)
    if name == "one_batch":         # fewer samples than one wave
        return wl.problem([6, 5, 7], [1, 2, 2, 1], 41, 44, name=name, init_rel=0.1)
    if name == "sparse_middle":     # most middle slices unobserved
        return wl.problem([12, 500, 14], [1, 2, 2, 1], 300, 45, name=name, init_rel=0.1)
    if name == "many_chunks":       # n = 300, rank 2, 1,000,000 samples: hundreds of chunks
        return wl.problem([300, 300, 300], [1, 2, 2, 1], 1_000_000, 46, name=name, init_rel=0.1)
    raise KeyError(name)


CASES = ["long_segments", "short_segments", "ragged_r3", "one_batch", "sparse_middle", "many_chunks"]


def observed(pb):
    return tt.tt_eval(pb.truth, pb.indices) + pb.noise_std * pb.noise


@pytest.mark.parametrize("name", CASES)
def test_low_rank_order3_pass_fp64_is_exact_and_repeatable(L, name):
    pb = case(name)
    say("case", name, pb.shape, pb.ranks, pb.n_obs)
    y = observed(pb)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, stop_rule="none", max_iter=0)
    try:
        cores = s.cores()
        g1, s1, rsq1 = s.sampled_pass()
        g2, s2, rsq2 = s.sampled_pass()
    finally:
        s.close()
    r = prgd.residual(cores, pb.indices, y)
    ref_g = prgd.core_gradient(cores, pb.indices, r)
    ref_s = prgd.slice_norms(pb.indices, r, pb.shape)
    assert abs(rsq1 - float(r @ r)) <= 1e-12 * float(r @ r)
    for k in range(3):
        scale = np.abs(ref_g[k]).max()
        assert np.abs(g1[k] - ref_g[k]).max() <= 1e-12 * scale, k
        np.testing.assert_allclose(s1[k], ref_s[k], rtol=1e-12, atol=1e-14 * ref_s[k].max())
        assert np.array_equal(g1[k], g2[k]) and np.array_equal(s1[k], s2[k]), k
    assert rsq1 == rsq2


@pytest.mark.parametrize("name", ["long_segments", "short_segments", "ragged_r3"])
def test_low_rank_order3_pass_mixed(L, name):
    pb = case(name)
    say("case", name)
    y = observed(pb)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, precision="mixed", stop_rule="none", max_iter=0)
    try:
        cores = s.cores()
        g, ss, rsq = s.sampled_pass()
        g2, ss2, _ = s.sampled_pass()
    finally:
        s.close()
    r = prgd.residual(cores, pb.indices, y)
    ref_g = prgd.core_gradient(cores, pb.indices, r)
    ref_s = prgd.slice_norms(pb.indices, r, pb.shape)
    bound_g = prgd.core_gradient([np.abs(c) for c in cores], pb.indices, np.abs(r))
    assert abs(rsq - float(r @ r)) <= 1e-5 * float(r @ r)
    for k in range(3):
        assert np.all(np.abs(g[k] - ref_g[k]) <= 4e-6 * 3 * bound_g[k] + 1e-30), k
        np.testing.assert_allclose(ss[k], ref_s[k], rtol=3e-5, atol=1e-12 * ref_s[k].max())
        assert np.array_equal(g[k], g2[k]) and np.array_equal(ss[k], ss2[k]), k


def test_low_rank_order3_iterates_match_reference(L):
    pb = case("ragged_r3")
    y = observed(pb)
    pol = prgd.Policy(step_rule="theory", c=0.8)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, step=0.8, stop_rule="none", max_iter=6)
    ref = [c.copy() for c in pb.init]
    try:
        for it in range(6):
            s.iterate(1)
            ref, _ = prgd.prgd_step(ref, pb.indices, y, pol, pb.ranks)
            d = tt.tt_dist(s.cores(), ref) / tt.tt_norm(ref)
            say(f"  iteration {it}: {d:.3e}")
            assert d <= 1e-10, (it, d)
    finally:
        s.close()
