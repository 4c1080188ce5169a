"""Python binding of librgg (include/rgg.h): argument marshalling only.

Every function keeps the C name.  Host arrays are numpy arrays; device
buffers are torch tensors on the library's device (torch supplies device
memory and streams, nothing else).  Every step of an update runs in librgg's
HIP kernels; if the library is not built this module raises on import of the
library, and no Python fallback exists.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  -- loads torch's HIP runtime before librgg so both share one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgg.so")

RGG_OK = 0
RGG_E_INVALID_ARG = -1
RGG_E_OUT_OF_MEMORY = -2
RGG_E_STATE_MISMATCH = -3
RGG_E_CAPACITY = -4
RGG_E_DEVICE = -5
RGG_E_UNSUPPORTED = -6
RGG_E_BUSY = -7

RGG_SE2, RGG_SE3, RGG_PLANAR_ARM = 0, 1, 2
RGG_GREEN, RGG_GRAY, RGG_RED = 0, 1, 2
RGG_PREC_FP64, RGG_PREC_FP32_RECHECK = 0, 1
RGG_INLINE_ALL, RGG_INLINE_NONE = 0, -1
RGG_VERDICT_FREE, RGG_VERDICT_COLLIDES, RGG_VERDICT_UNRESOLVED, RGG_VERDICT_BAD_ID = 0, 2, 3, 255
RGG_VALIDATE_DEFAULT_LEVELS, RGG_VALIDATE_DEFAULT_ACTIVE = 24, 256


class RggError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"librgg status {status}: {message}")
        self.status = status


class rgg_box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class rgg_robot(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_spheres", C.c_int32), ("n_links", C.c_int32),
                ("reserved", C.c_int32), ("sphere_pos", C.c_void_p), ("sphere_link", C.c_void_p),
                ("sphere_radius", C.c_void_p), ("link_length", C.c_void_p),
                ("base", C.c_double * 2)]


class rgg_roadmap_desc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("q", C.c_void_p), ("n_edges", C.c_int64),
                ("edge_uv", C.c_void_p)]


class rgg_build_opts(C.Structure):
    _fields_ = [("resolution", C.c_double), ("samples_per_edge", C.c_int32),
                ("precision", C.c_int32), ("band_rel", C.c_double),
                ("n_obstacle_slots", C.c_int64), ("cell_size", C.c_double),
                ("host_threads", C.c_int32), ("retest_capacity", C.c_int32),
                ("item_edges", C.c_int32), ("outer_obb", C.c_int32), ("inner_splines", C.c_int32),
                ("spline_tol", C.c_double), ("pair_list_capacity", C.c_int32), ("inline_rounds", C.c_int32),
                ("mem_budget", C.c_int64)]


class rgg_update_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_changed", C.c_int32), ("n_gray", C.c_int64),
                ("n_candidate_edges", C.c_int64), ("n_pairs", C.c_int64),
                ("n_outer_hits", C.c_int64), ("n_rechecked", C.c_int64),
                ("n_cells_visited", C.c_int64), ("test_bytes", C.c_int64), ("item_bytes", C.c_int64),
                ("fp64_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rgg_roadmap_info(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("n_slots", C.c_int64), ("dim", C.c_int32),
                ("n_spheres", C.c_int32), ("n_sphere_samples", C.c_int64),
                ("grid_cells", C.c_int64 * 3), ("cell_size", C.c_double),
                ("grid_entries", C.c_int64), ("device_bytes", C.c_int64),
                ("build_seconds", C.c_double), ("item_edges", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["grid_cells"] = list(self.grid_cells)
        return d


TUNE_MAX_CANDIDATES = 32


class rgg_tune_report(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("item_edges", C.c_int32),
                ("cell_size", C.c_double), ("grid_cells", C.c_int64 * 3),
                ("us_per_update", C.c_double), ("us_before", C.c_double),
                ("cand_item_edges", C.c_int32 * TUNE_MAX_CANDIDATES),
                ("cand_cell_size", C.c_double * TUNE_MAX_CANDIDATES),
                ("cand_us", C.c_double * TUNE_MAX_CANDIDATES)]

    def as_dict(self):
        n = self.n_candidates
        return {"n_candidates": n, "item_edges": self.item_edges, "cell_size": self.cell_size,
                "grid_cells": list(self.grid_cells), "us_per_update": self.us_per_update,
                "us_before": self.us_before,
                "candidates": [{"item_edges": self.cand_item_edges[k],
                                "cell_size": self.cand_cell_size[k], "us": self.cand_us[k]}
                               for k in range(n)]}


class rgg_update_req(C.Structure):
    _fields_ = [("rm", C.c_void_p), ("m", C.c_int64), ("d_old", C.c_void_p),
                ("d_new", C.c_void_p), ("d_labels", C.c_void_p), ("d_gray", C.c_void_p),
                ("gray_cap", C.c_int64), ("d_result", C.c_void_p)]


class rgg_server_opts(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_queue", C.c_int32), ("max_batch", C.c_int32),
                ("reserved", C.c_int32), ("pool_bytes", C.c_int64)]


class rgg_request_timing(C.Structure):
    _fields_ = [("latency_us", C.c_double), ("queue_us", C.c_double), ("service_us", C.c_double),
                ("batch_size", C.c_int32), ("reserved", C.c_int32)]


class rgg_server_req(C.Structure):
    _fields_ = [("rm", C.c_void_p), ("m", C.c_int64), ("old_boxes", C.c_void_p), ("new_boxes", C.c_void_p),
                ("d_labels", C.c_void_p), ("d_gray", C.c_void_p), ("gray_cap", C.c_int64),
                ("validate", C.c_int32), ("d_verdict", C.c_void_p)]


RESULT_BYTES = C.sizeof(rgg_update_result)

#: every symbol include/rgg.h declares
EXPORTS = ["rgg_context_create", "rgg_context_destroy", "rgg_build", "rgg_destroy",
           "rgg_roadmap_info_get", "rgg_update", "rgg_update_async", "rgg_graph_create",
           "rgg_graph_launch", "rgg_graph_destroy", "rgg_batch_create", "rgg_batch_launch",
           "rgg_batch_launch_graph", "rgg_batch_destroy", "rgg_batch_timing_enable", "rgg_batch_timing_read",
           "rgg_update_batch", "rgg_update_batch_noalloc",
           "rgg_server_start",
           "rgg_server_submit", "rgg_server_poll", "rgg_server_poll_timing", "rgg_server_info", "rgg_server_stop", "rgg_labels", "rgg_gray_list",
           "rgg_timing_enable", "rgg_timing_read", "rgg_tune", "rgg_batch_tune", "rgg_save", "rgg_load",
           "rgg_validate", "rgg_validate_async",
           "rgg_debug_geometry", "rgg_debug_second_forms", "rgg_debug_read_file",
           "rgg_last_error", "rgg_version"]

_lib = None


def lib():
    """Loads librgg.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "rgg_context_create": (I32, [C.c_int, C.POINTER(P)]),
        "rgg_context_destroy": (None, [P]),
        "rgg_build": (I32, [P, P, P, P, C.POINTER(P)]),
        "rgg_destroy": (I32, [P]),
        "rgg_roadmap_info_get": (I32, [P, P]),
        "rgg_update": (I32, [P, I64, P, P, P, P, I64, P, P]),
        "rgg_update_async": (I32, [P, P, I64, P, P, P, P, I64, P]),
        "rgg_graph_create": (I32, [P, I32, P, C.POINTER(P)]),
        "rgg_graph_launch": (I32, [P, P]),
        "rgg_graph_destroy": (I32, [P]),
        "rgg_batch_create": (I32, [P, I32, P, C.POINTER(P)]),
        "rgg_batch_launch": (I32, [P, P, P]),
        "rgg_batch_launch_graph": (I32, [P, P, P]),
        "rgg_batch_destroy": (I32, [P]),
        "rgg_batch_timing_enable": (I32, [P, I32]),
        "rgg_batch_timing_read": (I32, [P, P, P]),
        "rgg_update_batch": (I32, [P, I32, P, P]),
        "rgg_update_batch_noalloc": (I32, [P, I32, P, P]),
        "rgg_server_start": (I32, [P, P, C.POINTER(P)]),
        "rgg_server_submit": (I32, [P, P, C.POINTER(C.c_uint64)]),
        "rgg_server_poll": (I32, [P, C.c_uint64, I32, C.POINTER(I32), P, C.POINTER(C.c_double)]),
        "rgg_server_stop": (I32, [P]),
        "rgg_server_poll_timing": (I32, [P, C.c_uint64, I32, C.POINTER(I32), P, P]),
        "rgg_server_info": (I32, [P, P, C.POINTER(I64)]),
        "rgg_labels": (I32, [P, P]),
        "rgg_gray_list": (I32, [P, P, I64, P]),
        "rgg_timing_enable": (I32, [P, I32]),
        "rgg_timing_read": (I32, [P, P, P]),
        "rgg_tune": (I32, [P, I64, P, I32, P, I32, P]),
        "rgg_batch_tune": (I32, [P, P, P, I32, P]),
        "rgg_save": (I32, [P, C.c_char_p]),
        "rgg_validate": (I32, [P, P, I64, I32, I32, P, P, P]),
        "rgg_validate_async": (I32, [P, P, P, I64, P, I32, I32, P, P, P, P]),
        "rgg_load": (I32, [P, C.c_char_p, C.POINTER(P)]),
        "rgg_debug_geometry": (I32, [P, P, P, I64, I64, P, P, P, P]),
        "rgg_debug_second_forms": (I32, [P, P, P, I64, I64, P, P, P]),
        "rgg_debug_read_file": (I32, [C.c_char_p, C.POINTER(I64)]),
        "rgg_last_error": (C.c_char_p, []),
        "rgg_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st):
    if st != RGG_OK:
        raise RggError(st, lib().rgg_last_error().decode())
    return st


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# marshalling of robots, roadmaps and options
# --------------------------------------------------------------------------

class _Keep:
    """Holds the numpy arrays a C struct points into."""

    def __init__(self):
        self.arrays = []

    def f64(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.arrays.append(a)
        return a

    def i(self, a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        self.arrays.append(a)
        return a


def make_robot(robot, keep):
    """rgg_robot from an object with the fields of ``synth.Robot``."""
    r = rgg_robot()
    r.kind = robot.kind
    r.n_spheres = robot.sphere_radius.shape[0]
    r.n_links = 0 if robot.link_length is None else robot.link_length.shape[0]
    r.sphere_pos = _ptr(keep.f64(robot.sphere_pos))
    r.sphere_radius = _ptr(keep.f64(robot.sphere_radius))
    if robot.sphere_link is not None:
        r.sphere_link = _ptr(keep.i(robot.sphere_link, np.int32))
    if robot.link_length is not None:
        r.link_length = _ptr(keep.f64(robot.link_length))
    r.base[0], r.base[1] = float(robot.base[0]), float(robot.base[1])
    return r


def make_desc(q, edges, keep):
    d = rgg_roadmap_desc()
    qa = keep.f64(q)
    ea = keep.i(edges, np.int64)
    d.n_nodes = qa.shape[0]
    d.q = _ptr(qa)
    d.n_edges = ea.shape[0]
    d.edge_uv = _ptr(ea)
    return d


def make_opts(resolution=0.0, samples_per_edge=0, precision=RGG_PREC_FP64, band_rel=0.0,
              n_obstacle_slots=0, cell_size=0.0, host_threads=0, retest_capacity=0,
              item_edges=0, outer_obb=False, inner_splines=False, spline_tol=0.0, mem_budget=0,
              pair_list_capacity=0, inline_rounds=0):
    o = rgg_build_opts()
    o.mem_budget = mem_budget
    o.pair_list_capacity = pair_list_capacity
    o.inline_rounds = inline_rounds
    o.outer_obb = int(bool(outer_obb))
    o.inner_splines = int(bool(inner_splines))
    o.spline_tol = spline_tol
    o.resolution = resolution
    o.samples_per_edge = samples_per_edge
    o.precision = precision
    o.band_rel = band_rel
    o.n_obstacle_slots = n_obstacle_slots
    o.cell_size = cell_size
    o.host_threads = host_threads
    o.retest_capacity = retest_capacity
    o.item_edges = item_edges
    return o


def boxes_array(boxes):
    """(M, 6) float64 rows lo_x lo_y lo_z hi_x hi_y hi_z, the rgg_box layout."""
    a = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 6)
    return a


# --------------------------------------------------------------------------
# C entry points (same names)
# --------------------------------------------------------------------------

def rgg_context_create(device=0):
    h = C.c_void_p()
    _check(lib().rgg_context_create(device, C.byref(h)))
    return h


def rgg_context_destroy(ctx):
    lib().rgg_context_destroy(ctx)


def rgg_build(ctx, desc, robot, opts):
    h = C.c_void_p()
    _check(lib().rgg_build(ctx, C.byref(desc), C.byref(robot), C.byref(opts), C.byref(h)))
    return h


def rgg_destroy(rm):
    _check(lib().rgg_destroy(rm))


def rgg_roadmap_info_get(rm):
    info = rgg_roadmap_info()
    _check(lib().rgg_roadmap_info_get(rm, C.byref(info)))
    return info


def rgg_update(rm, old, new, n_edges, want_labels=True, gray_cap=None):
    """Host-buffer update.  Returns (labels or None, gray ids, n_gray, result)."""
    old = boxes_array(old)
    new = boxes_array(new)
    labels = np.empty(n_edges, dtype=np.uint8) if want_labels else None
    cap = n_edges if gray_cap is None else gray_cap
    gray = np.empty(max(cap, 1), dtype=np.int64)
    n = C.c_int64(0)
    res = rgg_update_result()
    st = lib().rgg_update(rm, old.shape[0], _ptr(old), _ptr(new), _ptr(labels), _ptr(gray), cap,
                          C.byref(n), C.byref(res))
    if st not in (RGG_OK, RGG_E_CAPACITY):
        _check(st)
    return labels, gray[:min(n.value, cap)].copy(), n.value, res


def rgg_update_async(rm, stream, m, d_old, d_new, d_labels, d_gray, gray_cap, d_result):
    """Device-buffer update queued on ``stream`` (a hipStream_t handle as int)."""
    _check(lib().rgg_update_async(rm, C.c_void_p(stream), m, _dptr(d_old), _dptr(d_new),
                                  _dptr(d_labels), _dptr(d_gray), gray_cap, _dptr(d_result)))


def rgg_labels(rm, n_edges):
    out = np.empty(max(n_edges, 1), dtype=np.uint8)
    _check(lib().rgg_labels(rm, _ptr(out)))
    return out[:n_edges]


def rgg_gray_list(rm, cap):
    out = np.empty(max(cap, 1), dtype=np.int64)
    n = C.c_int64(0)
    st = lib().rgg_gray_list(rm, _ptr(out), cap, C.byref(n))
    if st not in (RGG_OK, RGG_E_CAPACITY):
        _check(st)
    return out[:min(n.value, cap)].copy(), n.value


def rgg_graph_create(ctx, reqs):
    arr = (rgg_update_req * len(reqs))(*reqs)
    h = C.c_void_p()
    _check(lib().rgg_graph_create(ctx, len(reqs), arr, C.byref(h)))
    return h


def rgg_graph_launch(g, stream):
    _check(lib().rgg_graph_launch(g, C.c_void_p(stream)))


def rgg_graph_destroy(g):
    _check(lib().rgg_graph_destroy(g))


def rgg_batch_create(ctx, roadmaps):
    """roadmaps: handles (rgg_roadmap pointers) of distinct roadmaps."""
    arr = (C.c_void_p * len(roadmaps))(*[C.c_void_p(getattr(r, "value", r)) for r in roadmaps])
    h = C.c_void_p()
    _check(lib().rgg_batch_create(ctx, len(roadmaps), arr, C.byref(h)))
    return h


def rgg_batch_launch(b, reqs, stream):
    arr = (rgg_update_req * len(reqs))(*reqs)
    _check(lib().rgg_batch_launch(b, arr, C.c_void_p(stream)))


def rgg_batch_launch_graph(b, reqs, stream):
    arr = (rgg_update_req * len(reqs))(*reqs)
    _check(lib().rgg_batch_launch_graph(b, arr, C.c_void_p(stream)))


def rgg_batch_timing_enable(b, on):
    _check(lib().rgg_batch_timing_enable(b, 1 if on else 0))


def rgg_batch_timing_read(b):
    """(ms[6] summed per stage, launches timed) since the last read."""
    ms = np.zeros(6)
    n = C.c_int64(0)
    _check(lib().rgg_batch_timing_read(b, _ptr(ms), C.byref(n)))
    return ms, n.value


def rgg_batch_destroy(b):
    _check(lib().rgg_batch_destroy(b))


def rgg_update_batch(ctx, reqs, stream):
    arr = (rgg_update_req * len(reqs))(*reqs)
    _check(lib().rgg_update_batch(ctx, len(reqs), arr, C.c_void_p(stream)))


def rgg_update_batch_noalloc(ctx, reqs, stream):
    arr = (rgg_update_req * len(reqs))(*reqs)
    _check(lib().rgg_update_batch_noalloc(ctx, len(reqs), arr, C.c_void_p(stream)))


def rgg_server_start(ctx, n_streams=0, max_queue=0, max_batch=0, pool_bytes=0):
    o = rgg_server_opts(n_streams, max_queue, max_batch, 0, pool_bytes)
    h = C.c_void_p()
    _check(lib().rgg_server_start(ctx, C.byref(o), C.byref(h)))
    return h


def rgg_server_submit(srv, rm, old, new, d_labels=0, d_gray=0, gray_cap=0, validate=False, d_verdict=0):
    """Queues one update of roadmap handle `rm` (host box arrays [m, 6]);
    with ``validate`` the gray list is then validated and the gray labels
    rewritten (non-lazy).  Returns the ticket."""
    old = boxes_array(old)
    new = boxes_array(new)
    q = rgg_server_req(getattr(rm, "value", rm), old.shape[0], _ptr(old), _ptr(new), d_labels, d_gray, gray_cap,
                       1 if validate else 0, d_verdict)
    t = C.c_uint64()
    _check(lib().rgg_server_submit(srv, C.byref(q), C.byref(t)))
    return t.value


def rgg_server_poll(srv, ticket, wait=False):
    """(done, result, latency_us); result is None while the request runs."""
    done = C.c_int32()
    res = rgg_update_result()
    lat = C.c_double()
    _check(lib().rgg_server_poll(srv, ticket, 1 if wait else 0, C.byref(done), C.byref(res), C.byref(lat)))
    return (True, res, lat.value) if done.value else (False, None, 0.0)


def rgg_server_poll_timing(srv, ticket, wait=False):
    """(done, result, timing dict with latency_us, queue_us, service_us,
    batch_size); result and timing are None while the request runs."""
    done = C.c_int32()
    res = rgg_update_result()
    t = rgg_request_timing()
    _check(lib().rgg_server_poll_timing(srv, ticket, 1 if wait else 0, C.byref(done), C.byref(res), C.byref(t)))
    if not done.value:
        return False, None, None
    return True, res, {"latency_us": t.latency_us, "queue_us": t.queue_us, "service_us": t.service_us,
                       "batch_size": t.batch_size}


def rgg_server_info(srv):
    """The server's effective options and the free device memory at start."""
    o = rgg_server_opts()
    free = C.c_int64()
    _check(lib().rgg_server_info(srv, C.byref(o), C.byref(free)))
    return {"n_streams": o.n_streams, "max_queue": o.max_queue, "max_batch": o.max_batch,
            "pool_bytes": o.pool_bytes, "free_bytes_at_start": free.value}


def rgg_server_stop(srv):
    _check(lib().rgg_server_stop(srv))


def rgg_timing_enable(rm, on=True):
    _check(lib().rgg_timing_enable(rm, 1 if on else 0))


def rgg_timing_read(rm):
    ms = np.zeros(6)
    n = C.c_int64(0)
    _check(lib().rgg_timing_read(rm, _ptr(ms), C.byref(n)))
    return ms, n.value


def rgg_tune(rm, a, bs, reps=0):
    """Autotunes the roadmap's work decomposition on the updates a -> b -> a
    for each b in ``bs`` (one (M, 6) array, or a list of them); ``a`` must be
    the resident state.  Returns the report as a dict."""
    a = boxes_array(a)
    if isinstance(bs, np.ndarray) and bs.ndim == 2:
        bs = [bs]
    b = np.ascontiguousarray(np.concatenate([boxes_array(x) for x in bs]))
    rep = rgg_tune_report()
    _check(lib().rgg_tune(rm, a.shape[0], _ptr(a), len(bs), _ptr(b), int(reps), C.byref(rep)))
    return rep.as_dict()


def rgg_batch_tune(batch, a_list, b_list, reps=0):
    """Autotunes one work decomposition for every roadmap of ``batch`` on
    batched updates a[k] -> b[k] -> a[k] (lists in the batch's order)."""
    a_arr = [np.ascontiguousarray(boxes_array(x)) for x in a_list]
    b_arr = [np.ascontiguousarray(boxes_array(x)) for x in b_list]
    pa = (C.c_void_p * len(a_arr))(*[x.ctypes.data for x in a_arr])
    pb = (C.c_void_p * len(b_arr))(*[x.ctypes.data for x in b_arr])
    rep = rgg_tune_report()
    _check(lib().rgg_batch_tune(batch, pa, pb, int(reps), C.byref(rep)))
    return rep.as_dict()


def rgg_validate(rm, ids, max_level=0, max_active=0):
    """Full validation of edges ``ids`` against the resident obstacles:
    (verdict uint8, level int32, witness float64) arrays."""
    ids = np.ascontiguousarray(ids, dtype=np.int64).reshape(-1)
    n = ids.shape[0]
    verdict = np.zeros(max(n, 1), dtype=np.uint8)
    level = np.zeros(max(n, 1), dtype=np.int32)
    witness = np.zeros(max(n, 1), dtype=np.float64)
    _check(lib().rgg_validate(rm, _ptr(ids), n, int(max_level), int(max_active), _ptr(verdict), _ptr(level),
                              _ptr(witness)))
    return verdict[:n], level[:n], witness[:n]


def rgg_validate_async(rm, stream, d_ids, n, d_count, d_verdict, d_level, d_witness, max_level=0, max_active=0,
                       d_labels=None):
    """Device-buffer validation queued on ``stream``; ``d_count`` (a result
    tensor of an earlier update, or None) caps the count at its n_gray;
    ``d_labels`` (or None) receives GREEN / RED for the validated edges."""
    _check(lib().rgg_validate_async(rm, C.c_void_p(stream), _dptr(d_ids), int(n), _dptr(d_count),
                                    int(max_level), int(max_active), _dptr(d_verdict), _dptr(d_level),
                                    _dptr(d_witness), _dptr(d_labels)))


def rgg_save(rm, path):
    _check(lib().rgg_save(rm, os.fsencode(path)))


def rgg_load(ctx, path):
    h = C.c_void_p()
    _check(lib().rgg_load(ctx, os.fsencode(path), C.byref(h)))
    return h


def rgg_debug_geometry(desc, robot, opts, e0, e1):
    """Host build stage of edges [e0, e1): (n_configs, centres, capsules, boxes)."""
    L = lib()
    cnt = np.zeros(max(e1 - e0, 1), dtype=np.int64)
    _check(L.rgg_debug_geometry(C.byref(desc), C.byref(robot), C.byref(opts), e0, e1, _ptr(cnt),
                                None, None, None))
    cnt = cnt[:e1 - e0]
    B = robot.n_spheres
    D = 3 if robot.kind == RGG_SE3 else 2
    ctr = np.zeros((max(int(cnt.sum()), 1), B, D))
    cap = np.zeros((max(e1 - e0, 1), B, 2 * D + 1))
    box = np.zeros((max(e1 - e0, 1), 6), dtype=np.float32)
    _check(L.rgg_debug_geometry(C.byref(desc), C.byref(robot), C.byref(opts), e0, e1, _ptr(cnt),
                                _ptr(ctr), _ptr(cap), _ptr(box)))
    return cnt, ctr[:int(cnt.sum())], cap[:e1 - e0], box[:e1 - e0]


def rgg_debug_second_forms(desc, robot, opts, e0, e1):
    """Host build stage's oriented boxes [E, bodies, 2D + D*D] (or None) and
    spline segments: (counts [E, B], segments [sum, 2D + 1]) (or None)."""
    L = lib()
    E = e1 - e0
    B = robot.n_spheres
    D = 3 if robot.kind == RGG_SE3 else 2
    nb = robot.n_links if robot.kind == RGG_PLANAR_ARM else 1
    obb = np.zeros((max(E, 1), nb, 2 * D + D * D)) if opts.outer_obb else None
    cnt = np.zeros(max(E * B, 1), dtype=np.int64)
    _check(L.rgg_debug_second_forms(C.byref(desc), C.byref(robot), C.byref(opts), e0, e1, _ptr(obb),
                                    _ptr(cnt), None))
    spl = None
    if opts.inner_splines:
        seg = np.zeros((max(int(cnt[:E * B].sum()), 1), 2 * D + 1))
        _check(L.rgg_debug_second_forms(C.byref(desc), C.byref(robot), C.byref(opts), e0, e1, None, None,
                                        _ptr(seg)))
        spl = (cnt[:E * B].reshape(E, B), seg[:int(cnt[:E * B].sum())])
    return (obb[:E] if obb is not None else None), spl


def rgg_debug_read_file(path):
    """Reads and checks a roadmap file on the host as rgg_load does; returns
    its edge count."""
    n = C.c_int64(0)
    _check(lib().rgg_debug_read_file(os.fsencode(path), C.byref(n)))
    return n.value


def rgg_last_error():
    return lib().rgg_last_error().decode()


def rgg_version():
    return lib().rgg_version().decode()


# --------------------------------------------------------------------------
# convenience wrapper
# --------------------------------------------------------------------------

class Roadmap:
    """A roadmap resident on the GPU (wraps rgg_build / rgg_update / rgg_destroy)."""

    def __init__(self, ctx, robot, q, edges, n_slots, resolution=0.0, samples_per_edge=0,
                 precision=RGG_PREC_FP64, band_rel=0.0, cell_size=0.0, host_threads=0,
                 retest_capacity=0, item_edges=0, outer_obb=False, inner_splines=False, spline_tol=0.0,
                 mem_budget=0, pair_list_capacity=0, inline_rounds=0):
        keep = _Keep()
        self._keep = keep
        self.robot = make_robot(robot, keep)
        self.desc = make_desc(q, edges, keep)
        self.opts = make_opts(resolution, samples_per_edge, precision, band_rel, n_slots,
                              cell_size, host_threads, retest_capacity, item_edges, outer_obb,
                              inner_splines, spline_tol, mem_budget, pair_list_capacity, inline_rounds)
        self.h = rgg_build(ctx, self.desc, self.robot, self.opts)
        self.E = int(np.asarray(edges).shape[0])
        self.M = int(n_slots)

    @classmethod
    def from_workload(cls, ctx, w, precision=RGG_PREC_FP64, **kw):
        return cls(ctx, w.robot, w.q, w.edges, w.n_slots, w.resolution, w.samples_per_edge,
                   precision, **kw)

    def update(self, old, new, **kw):
        return rgg_update(self.h, old, new, self.E, **kw)

    def update_async(self, stream, d_old, d_new, d_labels, d_gray, d_result, gray_cap=None):
        cap = self.E if gray_cap is None else gray_cap
        rgg_update_async(self.h, stream, self.M, d_old, d_new, d_labels, d_gray, cap, d_result)

    def labels(self):
        return rgg_labels(self.h, self.E)

    def gray_list(self, cap=None):
        return rgg_gray_list(self.h, self.E if cap is None else cap)

    def info(self):
        return rgg_roadmap_info_get(self.h).as_dict()

    def tune(self, a, bs, reps=0):
        return rgg_tune(self.h, a, bs, reps)

    def validate(self, ids, max_level=0, max_active=0):
        return rgg_validate(self.h, ids, max_level, max_active)

    def save(self, path):
        rgg_save(self.h, path)

    @classmethod
    def load(cls, ctx, path):
        """A roadmap read back from a file rgg_save wrote."""
        self = cls.__new__(cls)
        self.h = rgg_load(ctx, path)
        info = rgg_roadmap_info_get(self.h)
        self.E, self.M = int(info.n_edges), int(info.n_slots)
        return self

    def close(self):
        if getattr(self, "h", None):
            rgg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def result_from_tensor(t):
    """Decodes an rgg_update_result held in a uint8 tensor (device or host)."""
    raw = t.detach().to("cpu").numpy().tobytes()
    return rgg_update_result.from_buffer_copy(raw[:RESULT_BYTES])
