"""The C ABI: the library loads, exports every declared symbol, and rejects invalid
problems on the host before any GPU work (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2501_13385_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "prgd.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(prgd_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(L.exported_symbols()) == syms


def test_cores_numel():
    assert L.prgd_cores_numel([10] * 4, [1, 2, 2, 2, 1]) == 120
    assert L.prgd_cores_numel([400] * 3, [1, 10, 10, 1]) == 48000
    assert L.prgd_cores_numel([3, 3], [2, 1, 1]) == -1


def _base():
    shape = [3, 3, 3]
    ranks = [1, 2, 2, 1]
    idx = np.array([[0, 1, 2], [0, 1, 2], [0, 0, 1]], dtype=np.int32)
    y = np.array([1.0, 2.0, 3.0])
    init = [np.ones((1, 3, 2)), np.ones((2, 3, 2)), np.ones((2, 3, 1))]
    return shape, ranks, idx, y, init


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a.update(ranks=[1, 5, 2, 1]), L.EINVAL),                     # rank above separation size
    (lambda a: a.update(ranks=[2, 2, 2, 1]), L.EINVAL),                     # r_0 != 1
    (lambda a: a.update(idx=np.array([[0, 1, 3], [0, 1, 2], [0, 0, 1]], dtype=np.int32)), L.EINVAL),
    (lambda a: a.update(idx=np.array([[0, 1, -1], [0, 1, 2], [0, 0, 1]], dtype=np.int32)), L.EINVAL),
    (lambda a: a.update(idx=np.array([[0, 1, 0], [0, 1, 0], [0, 0, 0]], dtype=np.int32)), L.EDUPLICATE),
    (lambda a: a.update(y=np.array([1.0, np.inf, 3.0])), L.EINVAL),
    (lambda a: a.update(kw={"step": -1.0}), L.EINVAL),
    (lambda a: a.update(kw={"step_policy": "const"}), L.EINVAL),           # const needs eps_fixed
    (lambda a: a.update(kw={"stop_rule": "error"}), L.EINVAL),             # needs truth
    (lambda a: a.update(kw={"tol": -1.0}), L.EINVAL),
    (lambda a: a.update(kw={"sort_mode": 3}), L.EINVAL),
])
def test_create_rejects_invalid_problems(mutate, code):
    shape, ranks, idx, y, init = _base()
    a = {"shape": shape, "ranks": ranks, "idx": idx, "y": y, "init": init, "kw": {}}
    mutate(a)
    init = a["init"]
    if a["ranks"] != ranks:
        r = a["ranks"]
        init = [np.ones((r[k], 3, r[k + 1])) for k in range(3)]
    with pytest.raises(L.PrgdError) as ei:
        L.prgd_create(a["shape"], a["ranks"], a["idx"], a["y"], init, **a["kw"])
    assert ei.value.status == code


def test_rank_above_build_limit_is_not_supported():
    shape = [20, 20, 20]
    ranks = [1, 17, 17, 1]
    idx = np.array([[0], [0], [0]], dtype=np.int32)
    init = [np.ones((ranks[k], 20, ranks[k + 1])) for k in range(3)]
    with pytest.raises(L.PrgdError) as ei:
        L.prgd_create(shape, ranks, idx, np.array([1.0]), init)
    assert ei.value.status == L.ENOTSUP


def test_status_strings_and_eval_validation():
    assert L.prgd_status_str(L.EDUPLICATE).startswith("duplicate")
    with pytest.raises(L.PrgdError):
        L.prgd_eval([3, 3], [1, 2, 1], [np.ones((1, 3, 2)), np.ones((2, 3, 1))],
                    np.array([[0], [5]], dtype=np.int32))


def test_server_rejects_bad_arguments_before_device_work():
    lib = L.load()
    d = L.prgd_server_desc()
    d.hbm_budget_bytes = 0
    d.max_slots = 0
    h = ctypes.c_void_p()
    assert lib.prgd_server_create(ctypes.byref(d), ctypes.byref(h)) == L.EINVAL
    assert lib.prgd_server_create(None, ctypes.byref(h)) == L.EINVAL
    t = ctypes.c_uint64(0)
    assert lib.prgd_server_submit(None, None, ctypes.byref(t)) == L.ESTATE
    assert lib.prgd_server_poll(None, 1, None, None, 0) == L.ESTATE
    assert lib.prgd_server_wait(None, 1, 0.0) == L.ESTATE
    assert lib.prgd_server_destroy(None) == L.ESTATE


def test_iteration_calls_reject_a_null_solver():
    lib = L.load()
    buf = (ctypes.c_double * L.NPHASES)()
    a, b = ctypes.c_double(1.0), ctypes.c_double(1.0)
    assert lib.prgd_iterate(None, 1) == L.ESTATE
    assert lib.prgd_iterate_profiled(None, 1, buf) == L.ESTATE
    assert lib.prgd_iterate_timed(None, 1, 1, ctypes.byref(a), ctypes.byref(b)) == L.ESTATE
    assert lib.prgd_sync(None) == L.ESTATE


def test_spectral_init_rejects_bad_arguments_before_device_work():
    shape, ranks = [4, 5, 6], [1, 2, 3, 1]
    idx = np.array([[0, 1], [2, 3], [4, 5]], dtype=np.int32)
    y = np.ones(2)
    g = np.zeros(sum(shape[k] * 5 for i in range(2) for k in range(i + 1, 3)))
    with pytest.raises(L.PrgdError) as e:
        L.prgd_spectral_init(shape, ranks, idx, y, g, 2)          # sketch below max rank
    assert e.value.status == L.EINVAL
    with pytest.raises(L.PrgdError) as e:
        L.prgd_spectral_init(shape, ranks, idx, y, g, 33)         # sketch above 32
    assert e.value.status == L.EINVAL
    bad = idx.copy()
    bad[2, 1] = 6
    with pytest.raises(L.PrgdError) as e:
        L.prgd_spectral_init(shape, ranks, bad, y, g, 5)          # index out of range
    assert e.value.status == L.EINVAL
    with pytest.raises(L.PrgdError) as e:
        L.prgd_spectral_init(shape, [1, 2, 17, 1], idx, y, g, 20)  # rank above 16
    assert e.value.status == L.ENOTSUP
    with pytest.raises(L.PrgdError) as e:
        L.prgd_spectral_init(shape, ranks, idx, np.array([1.0, np.nan]), g, 5)
    assert e.value.status == L.EINVAL


def test_create_rejects_a_bad_mode_interfaces_option():
    shape, ranks = [4, 5, 6, 3], [1, 2, 2, 2, 1]
    idx = np.array([[0, 1], [2, 3], [4, 5], [1, 2]], dtype=np.int32)
    init = [np.ones((ranks[k], shape[k], ranks[k + 1])) for k in range(4)]
    with pytest.raises(L.PrgdError) as e:
        L.Solver(shape, ranks, idx, np.ones(2), init, mode_interfaces=2)
    assert e.value.status == L.EINVAL


def test_duplicate_check_beyond_64_bit_linear_indices():
    """Five modes of 2^16: linear indices need 80 bits, so the 64-bit keys of
    (0,0,0,0,0) and (1,0,0,0,0) collide; distinct multi-indices with equal keys
    must pass the duplicate check and a true repeat must not."""
    shape, ranks = [1 << 16] * 5, [1, 1, 1, 1, 1, 1]
    init = [np.ones((1, 1 << 16, 1)) for _ in range(5)]
    colliding = np.array([[0, 1, 0], [0, 0, 1], [0, 0, 0], [0, 0, 0], [0, 0, 0]], dtype=np.int32)
    try:
        h = L.prgd_create(shape, ranks, colliding, np.ones(3), init)
        L.prgd_destroy(h)
    except L.PrgdError as e:       # no device here: later steps may fail, but not as duplicates
        assert e.status != L.EDUPLICATE
    repeated = np.array([[0, 1, 1], [0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0]], dtype=np.int32)
    with pytest.raises(L.PrgdError) as ei:
        L.prgd_create(shape, ranks, repeated, np.ones(3), init)
    assert ei.value.status == L.EDUPLICATE
