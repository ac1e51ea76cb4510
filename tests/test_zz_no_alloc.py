"""The entry point that allocates nothing (prgd_eval_noalloc) against
prgd_eval, through the C ABI: two calls in a row on device tensors, the second
with a smaller problem, each equal bit for bit to prgd_eval on the same inputs
(both run the same evaluation kernel on the same padded cores), plus the
refusal of cores larger than the fixed workspace."""
import sys

import numpy as np
import pytest

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


def run_noalloc(L, torch, pb):
    flat = L.pack(pb.truth)
    cd = torch.from_numpy(flat).to("cuda")
    idx = torch.from_numpy(np.ascontiguousarray(pb.indices, dtype=np.int32)).to("cuda")
    out = torch.full((pb.n_obs,), float("nan"), dtype=torch.float64, device="cuda")
    L.prgd_eval_noalloc(pb.shape, pb.ranks, cd, idx, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_eval_matches_eval_on_two_calls(L):
    import torch
    big = wl.problem([9, 12, 7, 10, 8], [1, 5, 9, 6, 4, 1], 50_000, 41, name="big", init_rel=0.1)
    small = wl.problem([5, 4, 6], [1, 3, 2, 1], 97, 42, name="small", init_rel=0.1)
    for pb in (big, small):
        say("case", pb.name, pb.shape, pb.ranks, pb.n_obs)
        got = run_noalloc(L, torch, pb)
        ref = L.prgd_eval(pb.shape, pb.ranks, pb.truth, pb.indices)
        assert np.array_equal(got, ref)


def test_noalloc_eval_refuses_cores_beyond_the_workspace(L):
    import torch
    # 2 x 40000 slices of 16 x 16 padded doubles: beyond 2^19 doubles
    shape, ranks = [40000, 40000], [1, 16, 1]
    flat = torch.zeros(2 * 40000 * 16, dtype=torch.float64, device="cuda")
    idx = torch.zeros((2, 4), dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PrgdError) as ei:
        L.prgd_eval_noalloc(shape, ranks, flat, idx, out)
    assert ei.value.status == L.ENOMEM
