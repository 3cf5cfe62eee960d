"""Thin ctypes binding of liblgt.so: the C ABI of include/lgt.h, same names.

Only argument marshalling happens here; every step of the evolution, the
reductions and the sampling run in the HIP library.  Importing this module
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgt.so")

LGT_OK, LGT_E_INVALID, LGT_E_UNSUPPORTED, LGT_E_OOM, LGT_E_DEVICE, LGT_E_STATE, LGT_E_BUSY = range(7)
LGT_C64, LGT_C128 = 0, 1
LGT_ORDER_TROTTER, LGT_ORDER_SYMMETRIC = 1, 2
LGT_FORM_FUSED, LGT_FORM_CIRCUIT, LGT_FORM_ANCILLA, LGT_FORM_CONTROLLED = 0, 1, 2, 3
LGT_INIT_PLUS, LGT_INIT_ZGROUND, LGT_INIT_BASIS, LGT_INIT_ZGROUND_CIRCUIT = 0, 1, 2, 3
LGT_GATE_H, LGT_GATE_X, LGT_GATE_RX, LGT_GATE_RZ, LGT_GATE_CNOT, LGT_GATE_CZ = range(6)
LGT_RAMP_PLAQ, LGT_RAMP_COUPLING, LGT_RAMP_EXPLICIT = 0, 1, 2
LGT_PLAN_NO_MERGE = 8
(LGT_OBS_NORM, LGT_OBS_Z, LGT_OBS_X, LGT_OBS_PLAQ, LGT_OBS_STAR, LGT_OBS_SIGMAX, LGT_OBS_SIGMAZ,
 LGT_OBS_ENERGY, LGT_OBS_ZDOS, LGT_OBS_XDOS) = range(10)

STATUS_NAMES = {0: "LGT_OK", 1: "LGT_E_INVALID", 2: "LGT_E_UNSUPPORTED", 3: "LGT_E_OOM",
                4: "LGT_E_DEVICE", 5: "LGT_E_STATE", 6: "LGT_E_BUSY"}

_dp = ctypes.POINTER(ctypes.c_double)


class lgt_schedule(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("n_steps", ctypes.c_int64), ("h_x", ctypes.c_double),
                ("h_p", ctypes.c_double), ("ramp", ctypes.c_int), ("g0", ctypes.c_double),
                ("g1", ctypes.c_double), ("s_rule", ctypes.c_int), ("cx", _dp), ("cz", _dp)]


class lgt_info_t(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("L", ctypes.c_int * 3), ("n_links", ctypes.c_int),
                ("n_plaq", ctypes.c_int), ("n_sites", ctypes.c_int), ("dtype", ctypes.c_int),
                ("state_bytes", ctypes.c_size_t), ("state", ctypes.c_void_p),
                ("stream", ctypes.c_void_p),
                ("plaq_masks", ctypes.POINTER(ctypes.c_uint64)),
                ("plaq_links", ctypes.POINTER(ctypes.c_int32)),
                ("star_masks", ctypes.POINTER(ctypes.c_uint64)),
                ("link_plaqs", ctypes.POINTER(ctypes.c_uint32)),
                ("n_qubits", ctypes.c_int)]


class lgt_observable(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_masks", ctypes.c_int),
                ("masks", ctypes.POINTER(ctypes.c_uint64)), ("cx", ctypes.c_double),
                ("cz", ctypes.c_double)]


class lgt_request(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("L", ctypes.c_int * 3), ("dtype", ctypes.c_int),
                ("sched", lgt_schedule), ("order", ctypes.c_int)]


class lgt_result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int), ("status", ctypes.c_int), ("energy", ctypes.c_double),
                ("plaq_mean", ctypes.c_double), ("gauss_violation", ctypes.c_double),
                ("norm", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double)]


class lgt_server_stats_t(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("used_bytes", ctypes.c_size_t),
                ("pending", ctypes.c_int), ("active", ctypes.c_int),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("undelivered", ctypes.c_uint64)]


# (name, restype, argtypes) of every exported entry point
_VP = ctypes.c_void_p
_SIGNATURES = [
    ("lgt_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    ("lgt_create_ex", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("lgt_destroy", ctypes.c_int, [_VP]),
    ("lgt_info", ctypes.c_int, [_VP, ctypes.POINTER(lgt_info_t)]),
    ("lgt_lattice_query", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_wilson_mask", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_line_mask", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_reset", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_uint64]),
    ("lgt_evolve", ctypes.c_int, [_VP, ctypes.POINTER(lgt_schedule), ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64]),
    ("lgt_measure", ctypes.c_int, [_VP, ctypes.POINTER(lgt_observable), _dp, ctypes.c_size_t]),
    ("lgt_sample", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_sample_noalloc", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_get_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("lgt_set_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("lgt_copy_state", ctypes.c_int, [_VP, _VP]),
    ("lgt_sync", ctypes.c_int, [_VP]),
    ("lgt_set_profiling", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lgt_kernel_stats", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64), _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    ("lgt_tune", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lgt_plan_describe", ctypes.c_int, [_VP, ctypes.c_char_p, ctypes.c_size_t]),
    ("lgt_plan_query", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]),
    ("lgt_set_plan", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lgt_thooft_mask", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_contour_mask", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_apply_pauli", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_uint64]),
    ("lgt_apply_gate", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
    ("lgt_set_graphs", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lgt_create_ancilla", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    ("lgt_critical_point", ctypes.c_int, [_dp, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp]),
    ("lgt_crossing", ctypes.c_int, [_dp, _dp, _dp, ctypes.c_int, _dp]),
    ("lgt_scan", ctypes.c_int, [_VP, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_size_t]),
    ("lgt_get_plan", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int)]),
    ("lgt_last_error", ctypes.c_char_p, [_VP]),
    ("lgt_batch_evolve", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP), ctypes.POINTER(lgt_schedule), ctypes.POINTER(ctypes.c_int), ctypes.c_int64, ctypes.c_int64]),
    ("lgt_batch_tune", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    ("lgt_batch_set_group", ctypes.c_int, [_VP, ctypes.c_int]),
    ("lgt_server_create", ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)]),
    ("lgt_server_submit", ctypes.c_int, [_VP, ctypes.POINTER(lgt_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("lgt_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(lgt_result)]),
    ("lgt_server_wait", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(lgt_result)]),
    ("lgt_server_destroy", ctypes.c_int, [_VP]),
    ("lgt_server_cancel", ctypes.c_int, [_VP, ctypes.c_uint64]),
    ("lgt_server_stats", ctypes.c_int, [_VP, ctypes.POINTER(lgt_server_stats_t)]),
    ("lgt_server_inject_fault", ctypes.c_int, [_VP, ctypes.c_uint64]),
]

_lib = None


def lib():
    """Load liblgt.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_1910_08020_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class LgtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int, ctx=None):
    if rc != LGT_OK:
        m = lib().lgt_last_error(ctx)
        raise LgtError(rc, m.decode() if m else "")


def _ints(L):
    return (ctypes.c_int * len(L))(*[int(x) for x in L])


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def lgt_create(d, L, periodic=1, dtype=LGT_C64):
    h = _VP()
    _check(lib().lgt_create(d, _ints(L), periodic, dtype, ctypes.byref(h)))
    return h


def lgt_create_ancilla(d, L, periodic=1, dtype=LGT_C64):
    h = _VP()
    _check(lib().lgt_create_ancilla(d, _ints(L), periodic, dtype, ctypes.byref(h)))
    return h


def lgt_create_ex(d, L, periodic, dtype, dev_buf: int, nbytes: int, stream: int | None):
    h = _VP()
    _check(lib().lgt_create_ex(d, _ints(L), periodic, dtype, _VP(dev_buf), nbytes,
                               _VP(stream) if stream else None, ctypes.byref(h)))
    return h


def lgt_destroy(ctx):
    _check(lib().lgt_destroy(ctx))


def lgt_info(ctx) -> dict:
    i = lgt_info_t()
    _check(lib().lgt_info(ctx, ctypes.byref(i)), ctx)
    return {
        "d": i.d, "L": list(i.L)[: i.d], "n_links": i.n_links, "n_qubits": i.n_qubits,
        "n_plaq": i.n_plaq,
        "n_sites": i.n_sites, "dtype": i.dtype, "state_bytes": i.state_bytes,
        "state": i.state, "stream": i.stream,
        "plaq_masks": np.array(i.plaq_masks[: i.n_plaq], dtype=np.uint64),
        "plaq_links": np.array(i.plaq_links[: 4 * i.n_plaq], dtype=np.int32).reshape(-1, 4),
        "star_masks": np.array(i.star_masks[: i.n_sites], dtype=np.uint64),
        "link_plaqs": np.array(i.link_plaqs[: i.n_links], dtype=np.uint32),
    }


def lgt_lattice_query(d, L) -> dict:
    nl, npq, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().lgt_lattice_query(d, _ints(L), ctypes.byref(nl), ctypes.byref(npq),
                                   ctypes.byref(ns), None, None))
    plaq = np.zeros(4 * npq.value, dtype=np.int32)
    stars = np.zeros(ns.value, dtype=np.uint64)
    _check(lib().lgt_lattice_query(d, _ints(L), None, None, None,
                                   plaq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   stars.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return {"n_links": nl.value, "n_plaq": npq.value, "n_sites": ns.value,
            "plaq_links": plaq.reshape(-1, 4), "star_masks": stars}


def lgt_wilson_mask(ctx, site, mu, nu, a, b) -> int:
    m = ctypes.c_uint64()
    _check(lib().lgt_wilson_mask(ctx, site, mu, nu, a, b, ctypes.byref(m)), ctx)
    return m.value


def lgt_line_mask(ctx, site, mu) -> int:
    m = ctypes.c_uint64()
    _check(lib().lgt_line_mask(ctx, site, mu, ctypes.byref(m)), ctx)
    return m.value


def lgt_reset(ctx, init=LGT_INIT_PLUS, basis_index=0):
    _check(lib().lgt_reset(ctx, init, basis_index), ctx)


def make_schedule(T, n_steps, h_x=1.0, h_p=1.0, ramp=LGT_RAMP_PLAQ, g0=0.0, g1=0.0, s_rule=0,
                  cx=None, cz=None) -> lgt_schedule:
    s = lgt_schedule(T=T, n_steps=n_steps, h_x=h_x, h_p=h_p, ramp=ramp, g0=g0, g1=g1,
                     s_rule=s_rule)
    if cx is not None:
        s._cx = np.ascontiguousarray(cx, dtype=np.float64)   # keep alive with the struct
        s._cz = np.ascontiguousarray(cz, dtype=np.float64)
        s.cx = s._cx.ctypes.data_as(_dp)
        s.cz = s._cz.ctypes.data_as(_dp)
    return s


def lgt_evolve(ctx, sched: lgt_schedule, order, form=LGT_FORM_FUSED, first_step=0, count=None):
    if count is None:
        count = sched.n_steps - first_step
    _check(lib().lgt_evolve(ctx, ctypes.byref(sched), order, form, first_step, count), ctx)


def lgt_measure(ctx, kind, masks=None, cx=0.0, cz=0.0, out_len=None) -> np.ndarray:
    o = lgt_observable(kind=kind, n_masks=0, cx=cx, cz=cz)
    keep = None
    if masks is not None:
        keep = np.ascontiguousarray(masks, dtype=np.uint64)
        o.n_masks = len(keep)
        o.masks = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    if out_len is None:
        out_len = max(64, len(keep) if keep is not None else 0)
    out = np.zeros(out_len)
    _check(lib().lgt_measure(ctx, ctypes.byref(o), out.ctypes.data_as(_dp), out_len), ctx)
    return out


def lgt_sample(ctx, n_shots, seed) -> np.ndarray:
    out = np.zeros(n_shots, dtype=np.uint64)
    _check(lib().lgt_sample(ctx, n_shots, seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), ctx)
    return out


def lgt_sample_noalloc(ctx, n_shots, seed) -> np.ndarray:
    out = np.zeros(n_shots, dtype=np.uint64)
    _check(lib().lgt_sample_noalloc(ctx, n_shots, seed,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), ctx)
    return out


def lgt_get_state(ctx, nbytes, dtype) -> np.ndarray:
    out = np.empty(nbytes // np.dtype(dtype).itemsize, dtype=dtype)
    _check(lib().lgt_get_state(ctx, out.ctypes.data_as(_VP), nbytes), ctx)
    return out


def lgt_set_state(ctx, arr: np.ndarray):
    arr = np.ascontiguousarray(arr)
    _check(lib().lgt_set_state(ctx, arr.ctypes.data_as(_VP), arr.nbytes), ctx)


def lgt_copy_state(dst, src):
    _check(lib().lgt_copy_state(dst, src), dst)


def lgt_sync(ctx):
    _check(lib().lgt_sync(ctx), ctx)


def lgt_set_profiling(ctx, on):
    """on: False/0 off, True/1 every launch, k > 1 every k-th launch per kernel family."""
    _check(lib().lgt_set_profiling(ctx, int(on)), ctx)


def lgt_kernel_stats(ctx) -> dict:
    cap = 32
    names = (ctypes.c_char_p * cap)()
    launches = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(lib().lgt_kernel_stats(ctx, names, launches, ms, cap, ctypes.byref(n)), ctx)
    return {names[i].decode(): (launches[i], ms[i]) for i in range(n.value)}


def lgt_tune(ctx, steps=8):
    _check(lib().lgt_tune(ctx, steps), ctx)


def lgt_plan_describe(ctx) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().lgt_plan_describe(ctx, buf, 512), ctx)
    return buf.value.decode()


def lgt_plan_query(n_links, dtype, plan=0) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().lgt_plan_query(n_links, dtype, plan, buf, 512), None)
    return buf.value.decode()


SCAN_COLUMNS = ("cx", "cz", "Z", "X", "norm")


def lgt_critical_point(g, h, stride=1):
    g = np.ascontiguousarray(g, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    gc, d2 = ctypes.c_double(), ctypes.c_double()
    _check(lib().lgt_critical_point(g.ctypes.data_as(_dp), h.ctypes.data_as(_dp), len(g), stride,
                                    ctypes.byref(gc), ctypes.byref(d2)), None)
    return gc.value, d2.value


def lgt_crossing(g, a, b):
    g = np.ascontiguousarray(g, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    gx = ctypes.c_double()
    _check(lib().lgt_crossing(g.ctypes.data_as(_dp), a.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                              len(g), ctypes.byref(gx)), None)
    return gx.value


def lgt_scan(ctx, sched: lgt_schedule, order, first_step, substeps, n_points, masks=None) -> np.ndarray:
    """Rows of (cx, cz, <Z>, <X>, norm, <W_0>, ...) after each block of `substeps`."""
    keep = None
    if masks is not None and len(masks):
        keep = np.ascontiguousarray(masks, dtype=np.uint64)
    nm = 0 if keep is None else len(keep)
    out = np.zeros((int(n_points), 5 + nm), dtype=np.float64)
    _check(lib().lgt_scan(ctx, ctypes.byref(sched), order, first_step, substeps, n_points,
                          None if keep is None else keep.ctypes.data, nm,
                          out.ctypes.data_as(_dp), out.size), ctx)
    return out


def lgt_thooft_mask(ctx, mu) -> int:
    m = ctypes.c_uint64()
    _check(lib().lgt_thooft_mask(ctx, mu, ctypes.byref(m)), ctx)
    return m.value


def lgt_contour_mask(ctx, k) -> int:
    m = ctypes.c_uint64()
    _check(lib().lgt_contour_mask(ctx, k, ctypes.byref(m)), ctx)
    return m.value


def lgt_apply_pauli(ctx, xmask=0, zmask=0):
    _check(lib().lgt_apply_pauli(ctx, xmask, zmask), ctx)


def lgt_apply_gate(ctx, gate, q0, q1=-1, angle=0.0):
    _check(lib().lgt_apply_gate(ctx, gate, q0, q1, angle), ctx)


def lgt_set_graphs(ctx, on: bool):
    _check(lib().lgt_set_graphs(ctx, 1 if on else 0), ctx)


def lgt_set_plan(ctx, plan: int):
    _check(lib().lgt_set_plan(ctx, plan), ctx)


def lgt_get_plan(ctx) -> int:
    p = ctypes.c_int()
    _check(lib().lgt_get_plan(ctx, ctypes.byref(p)), ctx)
    return p.value


def lgt_last_error(ctx=None) -> str:
    m = lib().lgt_last_error(ctx)
    return m.decode() if m else ""


def lgt_batch_evolve(ctxs, scheds, orders, first_step=0, count=None):
    n = len(ctxs)
    arr_c = (_VP * n)(*[c.value if isinstance(c, _VP) else c for c in ctxs])
    arr_s = (lgt_schedule * n)(*scheds)
    arr_o = (ctypes.c_int * n)(*orders)
    if count is None:
        count = scheds[0].n_steps - first_step
    _check(lib().lgt_batch_evolve(n, arr_c, arr_s, arr_o, first_step, count))


def lgt_batch_tune(ctxs, steps=8) -> int:
    n = len(ctxs)
    arr_c = (_VP * n)(*[c.value if isinstance(c, _VP) else c for c in ctxs])
    g = ctypes.c_int()
    _check(lib().lgt_batch_tune(n, arr_c, steps, ctypes.byref(g)))
    return g.value


def lgt_batch_set_group(ctx, group):
    _check(lib().lgt_batch_set_group(ctx, group), ctx)


def lgt_server_create(hbm_budget, max_slots, chunk_steps):
    h = _VP()
    _check(lib().lgt_server_create(hbm_budget, max_slots, chunk_steps, ctypes.byref(h)))
    return h


def lgt_server_submit(srv, req: lgt_request) -> int:
    t = ctypes.c_uint64()
    _check(lib().lgt_server_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def lgt_server_poll(srv, ticket) -> lgt_result:
    r = lgt_result()
    _check(lib().lgt_server_poll(srv, ticket, ctypes.byref(r)))
    return r


def lgt_server_wait(srv, ticket, timeout_ms=-1.0) -> lgt_result:
    r = lgt_result()
    _check(lib().lgt_server_wait(srv, ticket, timeout_ms, ctypes.byref(r)))
    return r


def lgt_server_destroy(srv):
    _check(lib().lgt_server_destroy(srv))


def lgt_server_cancel(srv, ticket):
    _check(lib().lgt_server_cancel(srv, ticket))


def lgt_server_stats(srv) -> dict:
    st = lgt_server_stats_t()
    _check(lib().lgt_server_stats(srv, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in lgt_server_stats_t._fields_}


def lgt_server_inject_fault(srv, ticket):
    _check(lib().lgt_server_inject_fault(srv, ticket))
