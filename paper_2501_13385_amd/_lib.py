"""ctypes binding of libprgd.so (include/prgd.h).  Argument marshalling only.

Every function named ``prgd_*`` here calls the C entry point of the same name;
all arithmetic of the method runs in the library's HIP kernels.  Importing
this module loads the library and raises if it has not been built.
"""

from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprgd.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
EINVAL, EDUPLICATE, ENOMEM, EDEVICE, EBREAKDOWN, ESTATE, ENOTSUP = -1, -2, -3, -4, -5, -6, -7
PREC = {"fp64": 0, "mixed": 1, "mixed_bf16": 2}
STEP = {"theory": 0, "const": 1, "adaptive": 2}
METRIC = {"data": 0, "euclidean": 1}
STOP = {"residual": 0, "change": 1, "error": 2, "none": 3}
PASS = {"auto": 0, "chain": 1, "modes": 2}


class PrgdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status}: {msg}")
        self.status = status


class prgd_desc(C.Structure):
    _fields_ = [
        ("order", C.c_int32),
        ("mode_sizes", C.POINTER(C.c_int32)),
        ("tt_ranks", C.POINTER(C.c_int32)),
        ("n_obs", C.c_int64),
        ("indices", C.c_void_p),
        ("values", C.c_void_p),
        ("values_fp64", C.c_int32),
        ("mem_device", C.c_int32),
        ("init_cores", C.POINTER(C.c_double)),
        ("truth_cores", C.POINTER(C.c_double)),
        ("precision", C.c_int32),
        ("step_policy", C.c_int32),
        ("step", C.c_double),
        ("eps_fixed", C.c_double),
        ("stop_rule", C.c_int32),
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
        ("sort_mode", C.c_int32),
        ("stream", C.c_void_p),
        ("metric", C.c_int32),
        ("mode_interfaces", C.c_int32),
        ("pass_kind", C.c_int32),
    ]


class prgd_iter_info(C.Structure):
    _fields_ = [
        ("iter", C.c_int32),
        ("flags", C.c_int32),
        ("rel_residual", C.c_double),
        ("rel_change", C.c_double),
        ("rel_error", C.c_double),
        ("eps", C.c_double),
        ("alpha", C.c_double),
    ]


class prgd_report(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("status", C.c_int32),
        ("rel_residual", C.c_double),
        ("rel_change", C.c_double),
        ("rel_error", C.c_double),
        ("seconds", C.c_double),
    ]


class prgd_server_desc(C.Structure):
    _fields_ = [
        ("hbm_budget_bytes", C.c_int64),
        ("max_slots", C.c_int32),
        ("iters_per_tick", C.c_int32),
    ]


class prgd_ticket_info(C.Structure):
    _fields_ = [
        ("report", prgd_report),
        ("submit_s", C.c_double),
        ("admit_s", C.c_double),
        ("finish_s", C.c_double),
        ("footprint_bytes", C.c_int64),
    ]


_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2501_13385_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    i32p = C.POINTER(C.c_int32)
    sig = {
        "prgd_cores_numel": (i64, [i32, i32p, i32p]),
        "prgd_create": (i32, [C.POINTER(prgd_desc), C.POINTER(vp)]),
        "prgd_iterate": (i32, [vp, i32]),
        "prgd_sync": (i32, [vp]),
        "prgd_iterate_profiled": (i32, [vp, i32, dp]),
        "prgd_iterate_timed": (i32, [vp, i32, i32, dp, dp]),
        "prgd_run": (i32, [vp, C.POINTER(prgd_report)]),
        "prgd_get_report": (i32, [vp, C.POINTER(prgd_report)]),
        "prgd_get_cores": (i32, [vp, dp, i64]),
        "prgd_get_history": (i32, [vp, C.POINTER(prgd_iter_info), i32, i32p]),
        "prgd_sampled_pass": (i32, [vp, dp, dp, dp]),
        "prgd_eval": (i32, [i32, i32p, i32p, dp, i64, vp, vp, i32, vp]),
        "prgd_spectral_init": (i32, [i32, i32p, i32p, i64, vp, vp, i32, vp, vp, vp]),
        "prgd_eval_noalloc": (i32, [i32, i32p, i32p, vp, i64, vp, vp, vp]),
        "prgd_destroy": (i32, [vp]),
        "prgd_status_str": (C.c_char_p, [i32]),
        "prgd_last_error": (C.c_char_p, []),
        "prgd_server_create": (i32, [C.POINTER(prgd_server_desc), C.POINTER(vp)]),
        "prgd_server_submit": (i32, [vp, C.POINTER(prgd_desc), C.POINTER(C.c_uint64)]),
        "prgd_server_poll": (i32, [vp, C.c_uint64, C.POINTER(prgd_ticket_info), dp, i64]),
        "prgd_server_wait": (i32, [vp, C.c_uint64, C.c_double]),
        "prgd_server_stats": (i32, [vp, i32p, i32p, i32p, C.POINTER(C.c_int64)]),
        "prgd_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    return [n for n in ("prgd_cores_numel", "prgd_create", "prgd_iterate", "prgd_iterate_profiled", "prgd_iterate_timed",
                        "prgd_sync", "prgd_run",
                        "prgd_get_report", "prgd_get_cores", "prgd_get_history", "prgd_sampled_pass",
                        "prgd_eval", "prgd_eval_noalloc", "prgd_spectral_init", "prgd_destroy", "prgd_status_str",
                        "prgd_last_error",
                        "prgd_server_create", "prgd_server_submit", "prgd_server_poll", "prgd_server_wait",
                        "prgd_server_stats", "prgd_server_destroy")]


def _check(st: int, allow=(OK,)) -> int:
    if st in allow:
        return st
    lib = load()
    raise PrgdError(st, f"{lib.prgd_status_str(st).decode()}: {lib.prgd_last_error().decode()}")


def _i32arr(v: Sequence[int]):
    a = (C.c_int32 * len(v))(*[int(x) for x in v])
    return a


def pack(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Packed layout of include/prgd.h: each core (r_{k-1}, n_k, r_k) in C order, concatenated."""
    return np.ascontiguousarray(np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cores]))


def unpack(flat: np.ndarray, shape: Sequence[int], ranks: Sequence[int]) -> List[np.ndarray]:
    out, p = [], 0
    for k in range(len(shape)):
        sz = ranks[k] * shape[k] * ranks[k + 1]
        out.append(flat[p:p + sz].reshape(ranks[k], shape[k], ranks[k + 1]).copy())
        p += sz
    return out


def prgd_cores_numel(shape: Sequence[int], ranks: Sequence[int]) -> int:
    return int(load().prgd_cores_numel(len(shape), _i32arr(shape), _i32arr(ranks)))


def prgd_status_str(st: int) -> str:
    return load().prgd_status_str(st).decode()


def prgd_last_error() -> str:
    return load().prgd_last_error().decode()


def _ptr_of(a):
    """Device pointer of a torch tensor, or host pointer of a numpy array."""
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr()), True
    return a.ctypes.data, False


def _make_desc(shape, ranks, indices, values, init_cores, *, truth_cores=None, precision="fp64",
               step_policy="theory", step=1.0, eps_fixed=0.0, stop_rule="residual", tol=1e-10,
               max_iter=500, sort_mode=-1, stream=None, metric="data", mode_interfaces=0,
               pass_kind="auto"):
    """prgd_desc for the arguments, plus the objects that must outlive the call."""
    m = len(shape)
    keep = []
    if hasattr(indices, "data_ptr"):
        assert indices.is_contiguous() and values.is_contiguous()
        n_obs = int(indices.shape[1])
        vfp64 = 1 if str(values.dtype) == "torch.float64" else 0
        ip, _ = _ptr_of(indices)
        vp_, _ = _ptr_of(values)
        mem_device = 1
    else:
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        values = np.ascontiguousarray(values)
        if values.dtype not in (np.float64, np.float32):
            values = values.astype(np.float64)
        keep += [indices, values]
        n_obs = int(indices.shape[1])
        vfp64 = 1 if values.dtype == np.float64 else 0
        ip, vp_ = indices.ctypes.data, values.ctypes.data
        mem_device = 0
    init = pack(init_cores)
    keep.append(init)
    truth = pack(truth_cores) if truth_cores is not None else None
    if truth is not None:
        keep.append(truth)
    ns, rs = _i32arr(shape), _i32arr(ranks)
    d = prgd_desc()
    d.order = m
    d.mode_sizes = ns
    d.tt_ranks = rs
    d.n_obs = n_obs
    d.indices = ip
    d.values = vp_
    d.values_fp64 = vfp64
    d.mem_device = mem_device
    d.init_cores = init.ctypes.data_as(C.POINTER(C.c_double))
    d.truth_cores = truth.ctypes.data_as(C.POINTER(C.c_double)) if truth is not None else None
    d.precision = PREC[precision]
    d.step_policy = STEP[step_policy]
    d.step = float(step)
    d.eps_fixed = float(eps_fixed)
    d.stop_rule = STOP[stop_rule]
    d.tol = float(tol)
    d.max_iter = int(max_iter)
    d.sort_mode = int(sort_mode)
    d.stream = stream
    d.metric = METRIC[metric]
    d.mode_interfaces = int(mode_interfaces)
    d.pass_kind = PASS[pass_kind]
    keep += [ns, rs]
    return d, keep


def prgd_create(shape, ranks, indices, values, init_cores, **kw):
    """Create a solver.  ``indices`` (m, N) int32 and ``values`` (N,) float64/float32 are numpy
    arrays (host) or torch CUDA tensors (device).  Returns an opaque handle (int)."""
    lib = load()
    d, keep = _make_desc(shape, ranks, indices, values, init_cores, **kw)
    h = C.c_void_p()
    _check(lib.prgd_create(C.byref(d), C.byref(h)))
    del keep
    return h.value


def prgd_iterate(h, iters: int) -> None:
    _check(load().prgd_iterate(h, int(iters)))


NPHASES = 6
PHASES = ["sampled_main", "sampled_finish", "project", "retract", "output", "truth"]


def prgd_iterate_profiled(h, iters: int) -> dict:
    """Run ``iters`` iterations with per-phase HIP events; returns summed milliseconds per phase."""
    buf = (C.c_double * NPHASES)()
    _check(load().prgd_iterate_profiled(h, int(iters), buf))
    return {PHASES[i]: float(buf[i]) for i in range(NPHASES)}


def prgd_iterate_timed(h, iters: int, stride: int = 1):
    """Run `iters` iterations; returns (mean ms of the main sampled kernel over
    the iterations it % stride == 0, whole run ms), device time."""
    k1 = C.c_double(0.0)
    tot = C.c_double(0.0)
    _check(load().prgd_iterate_timed(h, int(iters), int(stride), C.byref(k1), C.byref(tot)))
    return float(k1.value), float(tot.value)


def prgd_sync(h) -> None:
    _check(load().prgd_sync(h))


def _report(rep: prgd_report) -> dict:
    return {"iterations": rep.iterations, "status": rep.status, "rel_residual": rep.rel_residual,
            "rel_change": rep.rel_change, "rel_error": rep.rel_error, "seconds": rep.seconds}


def prgd_run(h) -> dict:
    rep = prgd_report()
    st = load().prgd_run(h, C.byref(rep))
    _check(st, allow=(OK, NOT_CONVERGED))
    return _report(rep)


def prgd_get_report(h) -> dict:
    rep = prgd_report()
    _check(load().prgd_get_report(h, C.byref(rep)))
    return _report(rep)


def prgd_get_cores(h, shape, ranks) -> List[np.ndarray]:
    numel = prgd_cores_numel(shape, ranks)
    out = np.empty(numel, dtype=np.float64)
    _check(load().prgd_get_cores(h, out.ctypes.data_as(C.POINTER(C.c_double)), numel))
    return unpack(out, shape, ranks)


def prgd_get_history(h, cap: int = 100000) -> List[dict]:
    buf = (prgd_iter_info * cap)()
    cnt = C.c_int32(0)
    _check(load().prgd_get_history(h, buf, cap, C.byref(cnt)))
    out = []
    for i in range(cnt.value):
        r = buf[i]
        rec = {"iter": r.iter, "rel_residual": r.rel_residual, "eps": r.eps, "alpha": r.alpha}
        if r.flags & 1:
            rec["rel_change"] = r.rel_change
        if r.flags & 2:
            rec["rel_error"] = r.rel_error
        out.append(rec)
    return out


def prgd_sampled_pass(h, shape, ranks):
    numel = prgd_cores_numel(shape, ranks)
    grad = np.empty(numel, dtype=np.float64)
    ssq = np.empty(int(sum(shape)), dtype=np.float64)
    rsq = C.c_double(0.0)
    _check(load().prgd_sampled_pass(h, grad.ctypes.data_as(C.POINTER(C.c_double)),
                                    ssq.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rsq)))
    splits = np.cumsum(shape)[:-1]
    return unpack(grad, shape, ranks), list(np.split(ssq, splits)), float(rsq.value)


def prgd_spectral_init(shape, ranks, indices, values, gauss, sketch, stream=None) -> List[np.ndarray]:
    """Sketched spectral initialisation on the GPU; host numpy in, list of cores out.

    ``gauss``: the standard-normal test matrices (see
    ``workloads.sketch_gaussians``), a list of arrays or one packed array.
    """
    lib = load()
    m = len(shape)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    val = np.ascontiguousarray(values, dtype=np.float64)
    if isinstance(gauss, np.ndarray) and gauss.ndim == 1:
        g = np.ascontiguousarray(gauss, dtype=np.float64)
    else:
        g = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in gauss]))
    numel = sum(int(ranks[k]) * int(shape[k]) * int(ranks[k + 1]) for k in range(m))
    out = np.empty(max(numel, 1), dtype=np.float64)
    _check(lib.prgd_spectral_init(m, _i32arr(shape), _i32arr(ranks), int(idx.shape[1]), idx.ctypes.data, val.ctypes.data,
                                  int(sketch), g.ctypes.data, out.ctypes.data, stream))
    return unpack(out, shape, ranks)


def prgd_eval(shape, ranks, cores, indices, out=None, stream=None):
    """TT values at the columns of ``indices``; numpy in -> numpy out, torch CUDA in -> torch CUDA out."""
    lib = load()
    flat = pack(cores)
    m = len(shape)
    if hasattr(indices, "data_ptr"):
        import torch
        n_obs = int(indices.shape[1])
        if out is None:
            out = torch.empty(n_obs, dtype=torch.float64, device=indices.device)
        _check(lib.prgd_eval(m, _i32arr(shape), _i32arr(ranks), flat.ctypes.data_as(C.POINTER(C.c_double)),
                             n_obs, int(indices.data_ptr()), int(out.data_ptr()), 1, stream))
        return out
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    n_obs = int(idx.shape[1])
    res = np.empty(n_obs, dtype=np.float64)
    _check(lib.prgd_eval(m, _i32arr(shape), _i32arr(ranks), flat.ctypes.data_as(C.POINTER(C.c_double)),
                         n_obs, idx.ctypes.data, res.ctypes.data, 0, stream))
    return res


def prgd_eval_noalloc(shape, ranks, cores_dev, indices_dev, out_dev, stream=None) -> None:
    """prgd_eval on device memory without allocating: ``cores_dev`` (packed float64),
    ``indices_dev`` (m, N) int32 and ``out_dev`` (N,) float64 are torch CUDA tensors.
    Queues the work on ``stream`` (a hipStream_t handle or None) and returns."""
    lib = load()
    m = len(shape)
    n_obs = int(indices_dev.shape[1])
    _check(lib.prgd_eval_noalloc(m, _i32arr(shape), _i32arr(ranks), int(cores_dev.data_ptr()), n_obs,
                                 int(indices_dev.data_ptr()), int(out_dev.data_ptr()), stream))


def prgd_destroy(h) -> None:
    _check(load().prgd_destroy(h))


class Solver:
    """Convenience owner of one solver handle (calls the functions above)."""

    def __init__(self, shape, ranks, indices, values, init_cores, **kw):
        self.shape = [int(s) for s in shape]
        self.ranks = [int(r) for r in ranks]
        self.h = prgd_create(self.shape, self.ranks, indices, values, init_cores, **kw)

    def iterate(self, k: int):
        prgd_iterate(self.h, k)

    def sync(self):
        prgd_sync(self.h)

    def iterate_profiled(self, k: int) -> dict:
        return prgd_iterate_profiled(self.h, k)

    def iterate_timed(self, k: int, stride: int = 1):
        return prgd_iterate_timed(self.h, k, stride)

    def run(self) -> dict:
        return prgd_run(self.h)

    def report(self) -> dict:
        return prgd_get_report(self.h)

    def cores(self) -> List[np.ndarray]:
        return prgd_get_cores(self.h, self.shape, self.ranks)

    def history(self) -> List[dict]:
        return prgd_get_history(self.h)

    def sampled_pass(self):
        return prgd_sampled_pass(self.h, self.shape, self.ranks)

    def close(self):
        if self.h:
            prgd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------------------
# request server
# ---------------------------------------------------------------------------

def prgd_server_create(hbm_budget_bytes: int = 0, max_slots: int = 256, iters_per_tick: int = 4):
    d = prgd_server_desc()
    d.hbm_budget_bytes = int(hbm_budget_bytes)
    d.max_slots = int(max_slots)
    d.iters_per_tick = int(iters_per_tick)
    h = C.c_void_p()
    _check(load().prgd_server_create(C.byref(d), C.byref(h)))
    return h.value


def prgd_server_submit(sv, shape, ranks, indices, values, init_cores, **kw) -> int:
    d, keep = _make_desc(shape, ranks, indices, values, init_cores, **kw)
    t = C.c_uint64(0)
    _check(load().prgd_server_submit(sv, C.byref(d), C.byref(t)))
    del keep
    return int(t.value)


def prgd_server_poll(sv, ticket: int, shape=None, ranks=None):
    """None while pending; else (status, info dict, cores or None) and the ticket is released."""
    info = prgd_ticket_info()
    out = None
    ptr, cap = None, 0
    if shape is not None:
        cap = prgd_cores_numel(shape, ranks)
        out = np.empty(cap, dtype=np.float64)
        ptr = out.ctypes.data_as(C.POINTER(C.c_double))
    st = load().prgd_server_poll(sv, C.c_uint64(ticket), C.byref(info), ptr, cap)
    if st == PENDING:
        return None
    if st == ESTATE or st == EINVAL:
        _check(st)
    res = _report(info.report)
    res.update({"submit_s": info.submit_s, "admit_s": info.admit_s, "finish_s": info.finish_s,
                "footprint_bytes": int(info.footprint_bytes)})
    cores = unpack(out, shape, ranks) if (out is not None and st >= 0) else None
    return st, res, cores


def prgd_server_wait(sv, ticket: int, timeout_s: float = -1.0) -> bool:
    st = load().prgd_server_wait(sv, C.c_uint64(ticket), float(timeout_s))
    if st == PENDING:
        return False
    _check(st)
    return True


def prgd_server_stats(sv) -> dict:
    q, l, f = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    b = C.c_int64(0)
    _check(load().prgd_server_stats(sv, C.byref(q), C.byref(l), C.byref(f), C.byref(b)))
    return {"queued": q.value, "live": l.value, "finished": f.value, "bytes_in_use": b.value}


def prgd_server_destroy(sv) -> None:
    _check(load().prgd_server_destroy(sv))


class Server:
    """Convenience owner of one request server."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 256, iters_per_tick: int = 4):
        self.h = prgd_server_create(hbm_budget_bytes, max_slots, iters_per_tick)
        self.meta = {}

    def submit(self, shape, ranks, indices, values, init_cores, **kw) -> int:
        t = prgd_server_submit(self.h, shape, ranks, indices, values, init_cores, **kw)
        self.meta[t] = ([int(s) for s in shape], [int(r) for r in ranks])
        return t

    def poll(self, ticket: int):
        shape, ranks = self.meta[ticket]
        res = prgd_server_poll(self.h, ticket, shape, ranks)
        if res is not None:
            del self.meta[ticket]
        return res

    def wait(self, ticket: int, timeout_s: float = -1.0) -> bool:
        return prgd_server_wait(self.h, ticket, timeout_s)

    def result(self, ticket: int, timeout_s: float = -1.0):
        if not self.wait(ticket, timeout_s):
            return None
        return self.poll(ticket)

    def stats(self) -> dict:
        return prgd_server_stats(self.h)

    def close(self):
        if self.h:
            prgd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
