"""ctypes binding of liblf2.so (include/lf2.h); argument marshalling only.

The functions here carry the C names and take plain integers for device
pointers and streams.  ``paper_1508_05610_amd.Plan`` wraps them for torch
tensors.  Loading fails loudly when the library has not been built: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblf2.so")

LF2_OK = 0
LF2_ERR_INVALID_ARG = -1
LF2_ERR_UNSUPPORTED = -2
LF2_ERR_OUT_OF_MEMORY = -3
LF2_ERR_DEVICE = -4
LF2_ERR_BUDGET = -5
LF2_ERR_BUSY = -6
LF2_ERR_NOT_READY = -7

LF2_R2C = 0
LF2_C2C = 1
LF2_FORWARD = -1
LF2_BACKWARD = 1

LF2_PLAN_AUTOTUNE = 0x10
LF2_IN_PLACE = 0x1
LF2_KLAYOUT_PAPER = 0x2
LF2_POISSON_CONTINUOUS_K2 = 0
LF2_POISSON_DISCRETE_K2 = 1
LF2_PK_OF_PHI = 2
LF2_NOALLOC_SCRATCH_BYTES = 128 << 20  # static workspace of lf2_poisson_solve_noalloc


class lf2_lattice(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("halo", ctypes.c_int32), ("size", ctypes.c_int64 * 3)]


class LF2Error(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        super().__init__(f"{func}: {status_string(status)} ({detail})")


class lf2_request(ctypes.Structure):
    _fields_ = [("lat", lf2_lattice), ("rho", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("dx", ctypes.c_double), ("flags", ctypes.c_uint32), ("nbins", ctypes.c_int32),
                ("d_pk", ctypes.c_void_p), ("d_kmean", ctypes.c_void_p),
                ("d_count", ctypes.c_void_p), ("t_arrival", ctypes.c_double)]


class lf2_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class lf2_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("rejected_busy", ctypes.c_int64),
                ("rejected_budget", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("bytes_in_flight", ctypes.c_size_t),
                ("peak_bytes_in_flight", ctypes.c_size_t), ("plans_cached", ctypes.c_int64),
                ("plan_hits", ctypes.c_int64), ("plan_misses", ctypes.c_int64),
                ("groups", ctypes.c_int64), ("grouped_requests", ctypes.c_int64),
                ("pooled_idle_bytes", ctypes.c_size_t), ("peak_bytes_in_use", ctypes.c_size_t),
                ("workspace_allocs", ctypes.c_int64), ("workspace_frees", ctypes.c_int64)]


_lib = None

# C signatures: name -> (restype, argtypes)
_vp, _i32, _u32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "lf2_fft_plan": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(lf2_lattice), _i32, _i32, _u32]),
    "lf2_fft_kspace": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "lf2_plan_workspace_bytes": (_i32, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "lf2_plan_get_tuning": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                   ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
    "lf2_plan_set_tuning": (_i32, [_vp, _i32, _i32, _i32]),
    "lf2_plan_get_schedule": (_i32, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32)]),
    "lf2_plan_set_schedule": (_i32, [_vp, _i32, ctypes.POINTER(_i32), _i32]),
    "lf2_plan_set_workspace": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "lf2_fft_execute": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "lf2_poisson_solve": (_i32, [_vp, _vp, _vp, _f64, _u32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "lf2_poisson_solve_noalloc": (_i32, [_vp, _vp, _vp, _f64, _u32, _i32, _vp, _vp, _vp, _vp,
                                         _vp]),
    "lf2_power_spectrum": (_i32, [_vp, _vp, _i32, _i32, _f64, _vp, _vp, _vp, _vp]),
    "lf2_plan_destroy": (_i32, [_vp]),
    "lf2_batch_plan": (_i32, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(lf2_lattice), _u32, _i32,
                              _f64, _u32]),
    "lf2_batch_execute": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 _vp]),
    "lf2_batch_error": (_i32, [_vp, ctypes.POINTER(_u32)]),
    "lf2_batch_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                              ctypes.POINTER(ctypes.c_size_t)]),
    "lf2_batch_destroy": (_i32, [_vp]),
    "lf2_batch_queues": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "lf2_server_create": (_i32, [ctypes.POINTER(_vp), ctypes.c_size_t, _i32, _i32, _i32]),
    "lf2_server_create_fake": (_i32, [ctypes.POINTER(_vp), ctypes.c_size_t, _i32, _i32, _u32,
                                      ctypes.c_uint64]),
    "lf2_server_prepare": (_i32, [_vp, _i32, ctypes.POINTER(lf2_lattice), _i32, _f64, _u32]),
    "lf2_server_submit": (_i32, [_vp, ctypes.POINTER(lf2_request), ctypes.POINTER(ctypes.c_uint64)]),
    "lf2_server_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(lf2_result), _i32]),
    "lf2_server_footprint": (_i32, [ctypes.POINTER(lf2_request), ctypes.POINTER(ctypes.c_size_t)]),
    "lf2_server_get_stats": (_i32, [_vp, ctypes.POINTER(lf2_server_stats)]),
    "lf2_server_destroy": (_i32, [_vp]),
    "lf2_server_now": (_f64, []),
    "lf2_update_halo": (_i32, [ctypes.POINTER(lf2_lattice), _i32, _i32, _vp, _vp]),
    "lf2_gradient": (_i32, [ctypes.POINTER(lf2_lattice), _i32, _vp, _vp, _f64, _vp]),
    "lf2_profile_enable": (_i32, [_i32]),
    "lf2_profile_reset": (_i32, []),
    "lf2_profile_count": (_i32, []),
    "lf2_profile_get": (_i32, [_i32, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_i64),
                                ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
    "lf2_status_string": (ctypes.c_char_p, [_i32]),
    "lf2_last_error": (ctypes.c_char_p, []),
    "lf2_version": (ctypes.c_char_p, []),
}


def exported_names():
    return list(_SIGS)


def load(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().lf2_status_string(status).decode()


def last_error() -> str:
    return load().lf2_last_error().decode()


def _check(status: int, func: str):
    if status != LF2_OK:
        raise LF2Error(status, func, last_error())


def lf2_version() -> str:
    return load().lf2_version().decode()


def lf2_fft_plan(sizes, halo: int, ncomp: int, kind: int, flags: int = 0) -> int:
    lat = lf2_lattice(3, int(halo), (ctypes.c_int64 * 3)(*[int(s) for s in sizes]))
    out = _vp()
    _check(load().lf2_fft_plan(ctypes.byref(out), ctypes.byref(lat), int(ncomp), int(kind),
                               int(flags)), "lf2_fft_plan")
    return out.value


def lf2_fft_plan_status(sizes, halo: int, ncomp: int, kind: int, flags: int = 0, dim: int = 3):
    """Raw status of lf2_fft_plan (for argument-validation tests); destroys any plan made."""
    lat = lf2_lattice(int(dim), int(halo), (ctypes.c_int64 * 3)(*[int(s) for s in sizes]))
    out = _vp()
    st = load().lf2_fft_plan(ctypes.byref(out), ctypes.byref(lat), int(ncomp), int(kind), int(flags))
    if st == LF2_OK and out.value:
        load().lf2_plan_destroy(out)
    return st


def lf2_fft_kspace(plan: int):
    ks = (_i64 * 3)()
    st = (_i64 * 3)()
    _check(load().lf2_fft_kspace(plan, ks, st), "lf2_fft_kspace")
    return tuple(ks), tuple(st)


def lf2_plan_get_tuning(plan: int, axis: int):
    """(variant, chunk, us_default, us_tuned) of the strided pass along axis."""
    v = _i32()
    c = _i32()
    a = _f64()
    b = _f64()
    _check(load().lf2_plan_get_tuning(plan, int(axis), ctypes.byref(v), ctypes.byref(c),
                                      ctypes.byref(a), ctypes.byref(b)), "lf2_plan_get_tuning")
    return int(v.value), int(c.value), float(a.value), float(b.value)


def lf2_plan_set_tuning(plan: int, axis: int, variant: int, chunk: int = 16):
    _check(load().lf2_plan_set_tuning(plan, int(axis), int(variant), int(chunk)),
           "lf2_plan_set_tuning")


def lf2_plan_get_schedule(plan: int, axis: int):
    """(radices tuple, runtime flag) of the passes along axis."""
    r = (_i32 * 15)()
    n = _i32()
    rt = _i32()
    _check(load().lf2_plan_get_schedule(plan, int(axis), r, ctypes.byref(n), ctypes.byref(rt)),
           "lf2_plan_get_schedule")
    return tuple(r[i] for i in range(n.value)), bool(rt.value)


def lf2_plan_set_schedule(plan: int, axis: int, radices):
    arr = (_i32 * 15)(*[int(v) for v in radices])
    _check(load().lf2_plan_set_schedule(plan, int(axis), arr, len(radices)),
           "lf2_plan_set_schedule")


def lf2_plan_workspace_bytes(plan: int) -> int:
    b = ctypes.c_size_t()
    _check(load().lf2_plan_workspace_bytes(plan, ctypes.byref(b)), "lf2_plan_workspace_bytes")
    return int(b.value)


def lf2_plan_set_workspace(plan: int, ptr: int, nbytes: int):
    _check(load().lf2_plan_set_workspace(plan, ptr or None, int(nbytes)), "lf2_plan_set_workspace")


def lf2_fft_execute(plan: int, direction: int, in_ptr: int, out_ptr: int, stream: int = 0):
    _check(load().lf2_fft_execute(plan, int(direction), in_ptr, out_ptr, stream or None),
           "lf2_fft_execute")


def lf2_poisson_solve(plan: int, rho_ptr: int, phi_ptr: int, dx: float, flags: int, nbins: int,
                      pk_ptr: int = 0, kmean_ptr: int = 0, count_ptr: int = 0,
                      parseval_ptr: int = 0, stream: int = 0):
    _check(load().lf2_poisson_solve(plan, rho_ptr, phi_ptr, float(dx), int(flags), int(nbins),
                                    pk_ptr or None, kmean_ptr or None, count_ptr or None,
                                    parseval_ptr or None, stream or None), "lf2_poisson_solve")


def lf2_power_spectrum(plan: int, field_ptr: int, field_is_kspace: int, nbins: int, dx: float,
                       pk_ptr: int = 0, kmean_ptr: int = 0, count_ptr: int = 0, stream: int = 0):
    _check(load().lf2_power_spectrum(plan, field_ptr, int(field_is_kspace), int(nbins), float(dx),
                                     pk_ptr or None, kmean_ptr or None, count_ptr or None,
                                     stream or None), "lf2_power_spectrum")


def lf2_plan_destroy(plan: int):
    _check(load().lf2_plan_destroy(plan), "lf2_plan_destroy")


LF2_BATCH_POISSON = 1
LF2_BATCH_PK = 2
LF2_BATCH_GROUPED = 4
LF2_BATCH_ONE_QUEUE = 8


def _lattices(sizes_list):
    arr = (lf2_lattice * len(sizes_list))()
    for i, s in enumerate(sizes_list):
        arr[i] = lf2_lattice(3, 0, (ctypes.c_int64 * 3)(*[int(v) for v in s]))
    return arr


def lf2_batch_plan(sizes_list, ops: int, nbins: int = 0, dx: float = 1.0,
                   poisson_flags: int = 0) -> int:
    out = _vp()
    lats = _lattices(sizes_list)
    _check(load().lf2_batch_plan(ctypes.byref(out), len(sizes_list), lats, int(ops), int(nbins),
                                 float(dx), int(poisson_flags)), "lf2_batch_plan")
    return out.value


def lf2_batch_queues(batch: int):
    """(queues of the persistent launch, 1 if each serves one XCD)."""
    n = _i32()
    x = _i32()
    _check(load().lf2_batch_queues(batch, ctypes.byref(n), ctypes.byref(x)), "lf2_batch_queues")
    return int(n.value), int(x.value)


def lf2_batch_plan_status(sizes_list, ops: int, nbins: int = 0, dx: float = 1.0,
                          poisson_flags: int = 0, halo: int = 0) -> int:
    """Raw status of lf2_batch_plan (argument-validation tests); destroys any batch made."""
    out = _vp()
    lats = _lattices(sizes_list)
    for i in range(len(sizes_list)):
        lats[i].halo = int(halo)
    st = load().lf2_batch_plan(ctypes.byref(out), len(sizes_list), lats, int(ops), int(nbins),
                               float(dx), int(poisson_flags))
    if st == LF2_OK and out.value:
        load().lf2_batch_destroy(out)
    return st


def _ptr_array(ptrs):
    if ptrs is None:
        return None
    return (_vp * len(ptrs))(*[p or None for p in ptrs])


def lf2_batch_execute(batch: int, rho_ptrs, phi_ptrs, pk_ptrs=None, kmean_ptrs=None,
                      count_ptrs=None, stream: int = 0):
    _check(load().lf2_batch_execute(batch, _ptr_array(rho_ptrs), _ptr_array(phi_ptrs),
                                    _ptr_array(pk_ptrs), _ptr_array(kmean_ptrs),
                                    _ptr_array(count_ptrs), stream or None), "lf2_batch_execute")


def lf2_batch_error(batch: int) -> int:
    e = _u32()
    _check(load().lf2_batch_error(batch, ctypes.byref(e)), "lf2_batch_error")
    return int(e.value)


def lf2_batch_info(batch: int):
    n = _i64()
    g = _i32()
    w = ctypes.c_size_t()
    _check(load().lf2_batch_info(batch, ctypes.byref(n), ctypes.byref(g), ctypes.byref(w)),
           "lf2_batch_info")
    return int(n.value), int(g.value), int(w.value)


def lf2_batch_destroy(batch: int):
    _check(load().lf2_batch_destroy(batch), "lf2_batch_destroy")


_lattice_cache: dict = {}


def make_request(sizes, rho_ptr: int, phi_ptr: int, dx: float = 1.0, flags: int = 0,
                 nbins: int = 0, pk_ptr: int = 0, kmean_ptr: int = 0, count_ptr: int = 0,
                 t_arrival: float = 0.0) -> lf2_request:
    # the lattice structs are cached per size (a request is built on every
    # submission, and its cost is part of the request's latency); pointer
    # fields take integers, 0 being NULL
    key = tuple(sizes)
    lat = _lattice_cache.get(key)
    if lat is None:
        lat = lf2_lattice(3, 0, (ctypes.c_int64 * 3)(*[int(v) for v in sizes]))
        if len(_lattice_cache) < 4096:
            _lattice_cache[key] = lat
    return lf2_request(lat, rho_ptr, phi_ptr, dx, flags, nbins, pk_ptr, kmean_ptr, count_ptr,
                       t_arrival)


def lf2_server_create(budget_bytes: int, max_slots: int, nstreams: int, max_queue: int) -> int:
    out = _vp()
    _check(load().lf2_server_create(ctypes.byref(out), int(budget_bytes), int(max_slots),
                                    int(nstreams), int(max_queue)), "lf2_server_create")
    return out.value


def lf2_server_create_fake(budget_bytes: int, max_slots: int, max_queue: int, delay_us: int,
                           fail_ticket: int = 0) -> int:
    out = _vp()
    _check(load().lf2_server_create_fake(ctypes.byref(out), int(budget_bytes), int(max_slots),
                                         int(max_queue), int(delay_us), int(fail_ticket)),
           "lf2_server_create_fake")
    return out.value


def lf2_server_prepare(server: int, sizes_list, nbins: int = 0, dx: float = 1.0, flags: int = 0):
    _check(load().lf2_server_prepare(server, len(sizes_list), _lattices(sizes_list), int(nbins),
                                     float(dx), int(flags)), "lf2_server_prepare")


def lf2_server_submit_status(server: int, req: lf2_request):
    """(status, ticket) of lf2_server_submit without raising (BUSY / BUDGET are normal)."""
    t = ctypes.c_uint64()
    st = load().lf2_server_submit(server, ctypes.byref(req), ctypes.byref(t))
    return st, int(t.value)


def lf2_server_poll(server: int, ticket: int, wait: bool = True):
    """None while the request runs (wait=False), else (status, t_arrival, t_admit, t_done)."""
    r = lf2_result()
    st = load().lf2_server_poll(server, int(ticket), ctypes.byref(r), int(bool(wait)))
    if st == LF2_ERR_NOT_READY:
        return None
    _check(st, "lf2_server_poll")
    return int(r.status), float(r.t_arrival), float(r.t_admit), float(r.t_done)


def lf2_server_footprint(req: lf2_request) -> int:
    b = ctypes.c_size_t()
    _check(load().lf2_server_footprint(ctypes.byref(req), ctypes.byref(b)), "lf2_server_footprint")
    return int(b.value)


def lf2_server_get_stats(server: int) -> dict:
    st = lf2_server_stats()
    _check(load().lf2_server_get_stats(server, ctypes.byref(st)), "lf2_server_get_stats")
    return {name: int(getattr(st, name)) for name, _ in lf2_server_stats._fields_}


def lf2_server_destroy(server: int):
    _check(load().lf2_server_destroy(server), "lf2_server_destroy")


def lf2_server_now() -> float:
    return float(load().lf2_server_now())


def lf2_update_halo(sizes, halo: int, ncomp: int, elem_bytes: int, field_ptr: int,
                    stream: int = 0):
    lat = lf2_lattice(3, int(halo), (ctypes.c_int64 * 3)(*[int(v) for v in sizes]))
    _check(load().lf2_update_halo(ctypes.byref(lat), int(ncomp), int(elem_bytes),
                                  field_ptr or None, stream or None), "lf2_update_halo")


def lf2_gradient(sizes, halo: int, ncomp: int, in_ptr: int, out_ptr: int, dx: float = 1.0,
                 stream: int = 0):
    lat = lf2_lattice(3, int(halo), (ctypes.c_int64 * 3)(*[int(v) for v in sizes]))
    _check(load().lf2_gradient(ctypes.byref(lat), int(ncomp), in_ptr or None, out_ptr or None,
                               float(dx), stream or None), "lf2_gradient")


def lf2_profile_enable(on: bool = True):
    _check(load().lf2_profile_enable(int(bool(on))), "lf2_profile_enable")


def lf2_profile_reset():
    _check(load().lf2_profile_reset(), "lf2_profile_reset")


def lf2_profile_count() -> int:
    return int(load().lf2_profile_count())


def lf2_profile_get(i: int):
    """(name, launches, total_ms, total_algorithmic_bytes) of kernel name i."""
    name = ctypes.create_string_buffer(128)
    n = _i64()
    ms = _f64()
    by = _f64()
    _check(load().lf2_profile_get(int(i), name, 128, ctypes.byref(n), ctypes.byref(ms),
                                  ctypes.byref(by)), "lf2_profile_get")
    return name.value.decode(), int(n.value), float(ms.value), float(by.value)


def profile_table():
    """{kernel name: (launches, total_ms, total_bytes)} of the records so far."""
    return {nm: (n, ms, by) for nm, n, ms, by in
            (lf2_profile_get(i) for i in range(lf2_profile_count()))}
