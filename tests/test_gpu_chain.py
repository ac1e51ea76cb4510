"""GPU parity of the one-pass chain kernel (orders >= 4, small mode sizes)
against the float64 reference, through the C ABI.

The chain kernel applies when every core from some split u on has a mode size
within one MFMA tile's slice range; the modes before u are shared by a whole
chunk of samples.  The cases cover u = 0, 1, 2 and 3, padded ranks 2, 4 and 8,
a first mode larger than the tile range (shared, so allowed), prefixes cut
into several chunks, a single partial batch, and float64 rank-8 chains of 4
unshared cores (the fewest the plan gives at rank 8) and of 8, 12 and 16,
whose right interfaces do not all fit the per-wave LDS slots and are parked
in segments.

Bars: sampled pass in float64 within 1e-12 of the reference (sums in another
order); iterates within 1e-10 per iteration; the pass repeats bit for bit
(no atomics); in mixed precision every gradient entry within
4e-6 * (sum over its samples of |R_j l_k[a] r_{k+1}[b]|) -- float32 rounding of the
chain (m - 1 products) and of the accumulation.
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


def rel_dist(a, b):
    return tt.tt_dist(a, b) / tt.tt_norm(b)


def chain_case(name):
    if name == "u0_r8":          # order 6, n = 4, ranks 8: one segment
        shape = [4] * 6
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 3000, 21, name=name, init_rel=0.1)
    if name == "u1_r8":          # order 7, n = 4: first mode shared per chunk
        shape = [4] * 7
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 9000, 22, name=name, init_rel=0.1)
    if name == "u2_r4":          # order 9, n = 3, ranks 4: two shared modes
        shape = [3] * 9
        return wl.problem(shape, wl.feasible_ranks(shape, 4), 12000, 23, name=name, init_rel=0.1)
    if name == "u1_r2_n16":      # padded rank 2, mode sizes up to 16
        shape = [16, 12, 16, 9, 14]
        return wl.problem(shape, [1, 2, 2, 2, 2, 1], 20000, 24, name=name, init_rel=0.1)
    if name == "u1_wide_first":  # the shared first mode has 40 slices (beyond one tile)
        shape = [40, 4, 4, 4, 4, 4, 4]
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 45000, 25, name=name, init_rel=0.1)
    if name == "u3_split":       # prefixes of ~1560 samples cut into several chunks
        shape = [4] * 9
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 100000, 26, name=name, init_rel=0.1)
    if name == "u1_r8_o9":       # order 9, n = 4, ranks 8, u = 1: eight unshared cores, the
        shape = [4] * 9          # right interfaces parked in two segments
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 9000, 31, name=name, init_rel=0.1)
    if name == "u0_r8_o12":      # order 12, u = 0: three segments
        shape = [4] * 12
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 2000, 32, name=name, init_rel=0.1)
    if name == "u0_r8_o16":      # order 16, u = 0: sixteen unshared cores, five segments
        shape = [4] * 16
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 3000, 33, name=name, init_rel=0.1)
    if name == "u0_r8_o4":       # order 4, rank 8, u = 0: the fewest unshared cores the plan
        shape = [4] * 4          # can give at rank 8 (two generic cores)
        return wl.problem(shape, wl.feasible_ranks(shape, 8), 200, 34, name=name, init_rel=0.1)
    if name == "tiny":           # fewer samples than one wave
        shape = [4, 3, 4, 3]
        return wl.problem(shape, [1, 3, 4, 3, 1], 20, 27, name=name, init_rel=0.1)
    if name == "ragged_r4":      # uneven ranks padded to 4, mode sizes 2..11
        shape = [5, 2, 11, 3, 7, 4]
        return wl.problem(shape, [1, 3, 4, 3, 4, 2, 1], 5000, 28, name=name, init_rel=0.1)
    raise KeyError(name)


CASES = ["u0_r8", "u1_r8", "u2_r4", "u1_r2_n16", "u1_wide_first", "u3_split", "tiny", "ragged_r4", "u1_r8_o9",
         "u0_r8_o12", "u0_r8_o16", "u0_r8_o4"]


def observed(pb):
    return tt.tt_eval(pb.truth, pb.indices) + pb.noise_std * pb.noise


def reference_pass(cores, pb, y):
    r = prgd.residual(cores, pb.indices, y)
    return r, prgd.core_gradient(cores, pb.indices, r), prgd.slice_norms(pb.indices, r, pb.shape)


@pytest.mark.parametrize("name", CASES)
def test_chain_sampled_pass_fp64(L, name):
    pb = chain_case(name)
    say("case", name, pb.shape, pb.ranks, pb.n_obs)
    y = observed(pb)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, stop_rule="none", max_iter=0, pass_kind="chain")
    try:
        cores = s.cores()
        g1, s1, rsq1 = s.sampled_pass()
        g2, s2, rsq2 = s.sampled_pass()
    finally:
        s.close()
    r, ref_g, ref_s = reference_pass(cores, pb, y)
    assert abs(rsq1 - float(r @ r)) <= 1e-12 * float(r @ r)
    for k in range(pb.order):
        scale = np.abs(ref_g[k]).max()
        assert np.abs(g1[k] - ref_g[k]).max() <= 1e-12 * scale, k
        np.testing.assert_allclose(s1[k], ref_s[k], rtol=1e-12, atol=1e-14 * ref_s[k].max())
        # no atomics: a second pass gives the same bits
        assert np.array_equal(g1[k], g2[k]) and np.array_equal(s1[k], s2[k]), k
    assert rsq1 == rsq2


@pytest.mark.parametrize("name", ["u1_r8", "u2_r4", "u1_wide_first", "ragged_r4"])
def test_chain_sampled_pass_mixed(L, name):
    pb = chain_case(name)
    say("case", name)
    y = observed(pb)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, precision="mixed", stop_rule="none", max_iter=0,
                 pass_kind="chain")
    try:
        cores = s.cores()
        g, ss, rsq = s.sampled_pass()
    finally:
        s.close()
    r, ref_g, ref_s = reference_pass(cores, pb, y)
    # entrywise bound: sum over the samples of |R_j| |l| |r| (the gradient of |R|
    # with the absolute cores), times float32 rounding of the chain and the sums
    abs_cores = [np.abs(c) for c in cores]
    bound_g = prgd.core_gradient(abs_cores, pb.indices, np.abs(r))
    assert abs(rsq - float(r @ r)) <= 1e-5 * float(r @ r)
    for k in range(pb.order):
        assert np.all(np.abs(g[k] - ref_g[k]) <= 4e-6 * pb.order * bound_g[k] + 1e-30), k
        np.testing.assert_allclose(ss[k], ref_s[k], rtol=1e-5 * pb.order, atol=1e-12 * ref_s[k].max())


@pytest.mark.parametrize("name,iters", [("u1_r8", 6), ("u2_r4", 6), ("u1_wide_first", 5), ("ragged_r4", 6),
                                        ("u1_r8_o9", 5), ("u0_r8_o12", 4)])
def test_chain_iterates_match_reference(L, name, iters):
    pb = chain_case(name)
    say("case", name)
    y = observed(pb)
    pol = prgd.Policy(step_rule="theory", c=0.8)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, step=0.8, stop_rule="none", max_iter=iters,
                 pass_kind="chain")
    ref = [c.copy() for c in pb.init]
    try:
        for it in range(iters):
            s.iterate(1)
            got = s.cores()
            ref, _ = prgd.prgd_step(ref, pb.indices, y, pol, pb.ranks)
            d = rel_dist(got, ref)
            say(f"  iteration {it}: {d:.3e}")
            assert d <= 1e-10, (it, d)
    finally:
        s.close()


def test_chain_and_mode_passes_agree_on_the_order14_shape(L):
    # the order-14, n = 4 shape at a reduced sample count: both kernels, five iterates
    shape = [4] * 14
    ranks = wl.feasible_ranks(shape, 8)
    pb = wl.problem(shape, ranks, 300_000, 29, name="o14", core_std=[1.0 / np.sqrt(ranks[k + 1]) for k in range(14)],
                    init_rel=0.1)
    y = observed(pb)
    out = {}
    for kind in ("chain", "modes"):
        s = L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, step=1.001, stop_rule="none", max_iter=5,
                     pass_kind=kind)
        try:
            s.iterate(5)
            out[kind] = s.cores()
        finally:
            s.close()
    d = rel_dist(out["chain"], out["modes"])
    say("chain vs modes", d)
    assert d <= 1e-10


def test_chain_is_refused_where_it_does_not_apply(L):
    pb = wl.problem([30, 30, 30, 30], [1, 4, 4, 4, 1], 2000, 30, name="wide", init_rel=0.1)
    y = observed(pb)
    with pytest.raises(L.PrgdError) as ei:
        L.Solver(pb.shape, pb.ranks, pb.indices, y, pb.init, stop_rule="none", max_iter=0, pass_kind="chain")
    assert ei.value.status == L.ENOTSUP
