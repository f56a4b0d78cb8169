"""ctypes binding of liboctmg.so (C ABI in include/octmg.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  The library must have been built (``python -m
paper_2205_09411_amd.build``); there is no fallback, and importing a missing
library raises.  PyTorch is optional here: device tensors and streams may be
passed by pointer (``tensor.data_ptr()``, ``torch.cuda.current_stream()``).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboctmg.so")

OK = 0
ERR_INVALID, ERR_OOM, ERR_HIP, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_GEOMETRY, ERR_BUDGET = -1, -2, -3, -4, -5, -6, -7
LSF_NONE, LSF_SPHERES, LSF_CYLINDER_Z = 0, 1, 2
LSF_CALLBACK = 8
# double f(const double *x, void *user): a level set given as a host function
LSF_FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)
REFINE_UNIFORM, REFINE_NEAR_INTERFACE = 0, 1
FP64, MIXED = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
CYCLE_V, CYCLE_FMG = 0, 1
FIELD_PHI, FIELD_G, FIELD_OLD = 0, 1, 2
STEP_HALF_SWEEP, STEP_SMOOTH, STEP_RESTRICT_FAS, STEP_PROLONG, STEP_COARSE_SOLVE, STEP_RESTRICT_RHS = range(6)


class OctmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"octmg status {status}: {msg}")
        self.status = status


class GeomDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("block_n", C.c_int), ("max_level", C.c_int), ("refine_kind", C.c_int),
                ("lsf_kind", C.c_int), ("lsf_n", C.c_int), ("coarse_n", C.c_int), ("neumann_faces", C.c_int),
                ("refine_width", C.c_double), ("eps_tol", C.c_double), ("mask_factor", C.c_double),
                ("w_min", C.c_double), ("lo", C.c_double * 3), ("lsf_params", C.POINTER(C.c_double)),
                ("uniform_level", C.c_int), ("reserved", C.c_int), ("lsf_fn", LSF_FN), ("lsf_user", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("cycle_kind", C.c_int), ("max_cycles", C.c_int), ("zero_start", C.c_int),
                ("graph_mode", C.c_int), ("rtol", C.c_double)]


class LaunchConfig(C.Structure):
    _fields_ = [("block_order", C.c_int), ("bottom_kind", C.c_int), ("bottom_max_blocks", C.c_int),
                ("graph_mode", C.c_int), ("pair_max_blocks", C.c_int), ("prolong_fused", C.c_int),
                ("red_preset", C.c_int), ("update_fused", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("r0", C.c_double), ("r_final", C.c_double),
                ("history", C.c_double * 64), ("rhs_status", C.POINTER(C.c_int)), ("rhs_cycles", C.POINTER(C.c_int)),
                ("rhs_r0", C.POINTER(C.c_double)), ("rhs_r_final", C.POINTER(C.c_double))]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_lanes", C.c_int), ("precision", C.c_int),
                ("max_cycles", C.c_int), ("reserved", C.c_int)]


class Result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int), ("cycles", C.c_int), ("r0", C.c_double),
                ("r_final", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "admitted", "completed", "failed", "states_created",
                                          "states_released", "cycles_launched", "lane_cycles", "peak_bytes",
                                          "bytes_in_use")] + [("now", C.c_double)]


_lib = None
_vp, _dp, _ip, _i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)
_SIGS = {
    "octmg_last_error": (C.c_char_p, []),
    "octmg_version": (C.c_int, []),
    "octmg_plan_levels": (C.c_int, [C.POINTER(GeomDesc), _ip, _i64p]),
    "octmg_plan_blocks": (C.c_int, [C.POINTER(GeomDesc), C.c_int, _ip, _ip]),
    "octmg_ctx_create": (C.c_int, [C.c_int, C.POINTER(Allocator), C.c_char_p, C.POINTER(_vp)]),
    "octmg_ctx_destroy": (None, [_vp]),
    "octmg_geom_create": (C.c_int, [C.POINTER(GeomDesc), C.c_int, C.POINTER(_vp)]),
    "octmg_geom_create_in": (C.c_int, [_vp, C.POINTER(GeomDesc), C.c_int, C.POINTER(_vp)]),
    "octmg_geom_destroy": (None, [_vp]),
    "octmg_geom_info": (C.c_int, [_vp, _i64p]),
    "octmg_geom_level_info": (C.c_int, [_vp, C.c_int, _i64p]),
    "octmg_geom_leaf_coords": (C.c_int, [_vp, _dp, _ip]),
    "octmg_geom_iface_points": (C.c_int, [_vp, _dp]),
    "octmg_geom_domain_points": (C.c_int, [_vp, _dp]),
    "octmg_geom_records": (C.c_int, [_vp, C.c_int, _ip, _dp, _dp]),
    "octmg_geom_block_positions": (C.c_int, [_vp, C.c_int, _ip, _ip]),
    "octmg_state_create": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(_vp)]),
    "octmg_state_destroy": (None, [_vp]),
    "octmg_state_set_smoothing": (C.c_int, [_vp, C.c_int, C.c_int]),
    "octmg_state_set_fused_levels": (C.c_int, [_vp, C.c_int]),
    "octmg_set_boundary": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "octmg_set_rhs": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp]),
    "octmg_set_solution": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp]),
    "octmg_get_solution": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp]),
    "octmg_zero_solution": (C.c_int, [_vp, _vp]),
    "octmg_cycle": (C.c_int, [_vp, C.c_int, C.c_int, _vp]),
    "octmg_residual_norm": (C.c_int, [_vp, C.c_int, _dp, _vp]),
    "octmg_gradient": (C.c_int, [_vp, C.c_int, _vp, C.c_int, _vp]),
    "octmg_solve": (C.c_int, [_vp, C.POINTER(SolveOpts), _vp, C.POINTER(SolveReport)]),
    "octmg_solve_noalloc": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(SolveOpts), _vp, C.POINTER(SolveReport)]),
    "octmg_geom_adapt": (C.c_int, [_vp, _vp, C.c_int, C.POINTER(_vp), _i64p]),
    "octmg_state_remap": (C.c_int, [_vp, _vp, _vp]),
    "octmg_state_set_launch": (C.c_int, [_vp, C.POINTER(LaunchConfig)]),
    "octmg_state_get_launch": (C.c_int, [_vp, C.POINTER(LaunchConfig)]),
    "octmg_autotune": (C.c_int, [_vp, C.POINTER(SolveOpts), C.c_int, _vp, C.POINTER(LaunchConfig), _dp, _ip]),
    "octmg_profile_enable": (C.c_int, [_vp, C.c_int]),
    "octmg_profile_read": (C.c_int, [_vp, _dp]),
    "octmg_debug_get_field": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp]),
    "octmg_debug_set_field": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp]),
    "octmg_debug_step": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _vp]),
    "octmg_server_create": (C.c_int, [C.c_int, C.POINTER(ServerOpts), C.POINTER(_vp)]),
    "octmg_server_add_geometry": (C.c_int, [_vp, _vp, _vp, _vp, _ip]),
    "octmg_server_submit": (C.c_int, [_vp, C.c_int, _vp, C.c_int, _vp, C.c_int, C.c_double,
                                      C.POINTER(C.c_uint64)]),
    "octmg_server_poll": (C.c_int, [_vp, C.POINTER(Result), C.c_int, _ip]),
    "octmg_server_get_stats": (C.c_int, [_vp, C.POINTER(ServerStats)]),
    "octmg_server_destroy": (None, [_vp]),
}


# Handles still open.  At interpreter exit they are closed in dependency
# order (servers, then states, then geometries) by an atexit hook registered
# when the library loads, so that no library object -- a server's worker
# thread, captured graphs, pinned host memory -- is still alive when the HIP
# runtime tears itself down after Python has finished; __del__ does nothing
# from then on.
_live = weakref.WeakSet()
_shutting_down = False


def close_all():
    """Close every open handle (servers, states, geometries)."""
    for kind in (Server, State, Geometry, Context):
        for obj in [o for o in list(_live) if isinstance(o, kind)]:
            try:
                obj.close()
            except Exception:
                pass


def _at_exit():
    global _shutting_down
    close_all()
    _shutting_down = True


def _finalizing() -> bool:
    return _shutting_down or sys.is_finalizing()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2205_09411_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        atexit.register(_at_exit)
    return _lib


def exported_names():
    return list(_SIGS)


def _check(status: int):
    if status != OK:
        raise OctmgError(status, lib().octmg_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def lsf_callback(f):
    """C level-set callback from a Python function f(x, y, z) -> float
    (keep the returned object alive as long as the geometry)."""
    return LSF_FN(lambda x, user: float(f(x[0], x[1], x[2])))


def make_desc(geom) -> GeomDesc:
    """GeomDesc from a workloads.Geometry-like object (keeps params and a
    level-set callback ``geom.lsf_fn`` alive)."""
    params = np.ascontiguousarray(np.asarray(geom.lsf_params, dtype=np.float64).reshape(-1))
    if params.size == 0:
        params = np.zeros(1)
    d = GeomDesc()
    d.dim, d.block_n, d.max_level = geom.dim, geom.block_n, geom.max_level
    d.refine_kind, d.lsf_kind, d.lsf_n = geom.refine_kind, geom.lsf_kind, geom.lsf_n
    d.coarse_n = geom.coarse_n
    d.neumann_faces = getattr(geom, "neumann_faces", 0)
    d.uniform_level = getattr(geom, "uniform_level", 0)
    d.refine_width, d.eps_tol, d.mask_factor, d.w_min = geom.refine_width, geom.eps_tol, geom.mask_factor, geom.w_min
    for i in range(3):
        d.lo[i] = geom.lo[i]
    d.lsf_params = _ptr(params, C.c_double)
    d._keep = params
    fn = getattr(geom, "lsf_fn", None)
    if fn is not None:
        cb = fn if isinstance(fn, LSF_FN) else lsf_callback(fn)
        d.lsf_fn = cb
        d._keep_fn = cb
    return d


def plan_levels(geom):
    """Host-only tree plan: list of dicts per level (no device needed)."""
    d = make_desc(geom)
    n = C.c_int()
    info = np.zeros(4 * 24, dtype=np.int64)
    _check(lib().octmg_plan_levels(C.byref(d), C.byref(n), _ptr(info, C.c_int64)))
    keys = ["n", "Nb", "nblocks", "nleaf"]
    return [dict(zip(keys, (int(v) for v in info[4 * i:4 * i + 4]))) for i in range(n.value)]


def plan_blocks(geom, level: int):
    d = make_desc(geom)
    nb = plan_levels(geom)[level]["nblocks"]
    pos = np.zeros((nb, 3), dtype=np.int32)
    leaf = np.zeros(nb, dtype=np.int32)
    _check(lib().octmg_plan_blocks(C.byref(d), level, _ptr(pos, C.c_int), _ptr(leaf, C.c_int)))
    return pos, leaf


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator (the
    library's buffers then show up in torch's memory statistics).  The
    callbacks may run on the library's worker threads."""

    def __init__(self):
        import threading
        self._blocks = {}
        self._lock = threading.Lock()

        def alloc(nbytes, device, user):
            import torch
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
            with self._lock:
                self._blocks[t.data_ptr()] = t
            return t.data_ptr()

        def free(ptr, nbytes, device, user):
            with self._lock:
                self._blocks.pop(ptr, None)

        self.c = Allocator(ALLOC_FN(alloc), FREE_FN(free), None)

    def bytes_held(self) -> int:
        with self._lock:
            return sum(t.numel() for t in self._blocks.values())


class Context:
    """Device, optional allocator (e.g. TorchAllocator()) and optional
    tune-cache file shared by the geometries created in it."""

    def __init__(self, device: int = 0, allocator=None, tune_cache: str = None):
        self.allocator = allocator  # kept alive for the callbacks
        self.device = device
        h = _vp()
        _check(lib().octmg_ctx_create(device, C.byref(allocator.c) if allocator is not None else None,
                                      tune_cache.encode() if tune_cache else None, C.byref(h)))
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().octmg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        if not _finalizing():
            self.close()


class Geometry:
    """Tree, FP64 interface setup and coarse inverse on one HIP device (or in
    a Context, whose allocator and tune cache it then uses)."""

    def __init__(self, geom, device: int = 0, _handle=None, ctx: "Context" = None):
        self.desc = make_desc(geom)
        self.geom = geom
        self.ctx = ctx  # a geometry keeps its context (and allocator callbacks) alive
        if ctx is not None:
            device = ctx.device
        if _handle is None:
            h = _vp()
            if ctx is not None:
                _check(lib().octmg_geom_create_in(ctx._h, C.byref(self.desc), device, C.byref(h)))
            else:
                _check(lib().octmg_geom_create(C.byref(self.desc), device, C.byref(h)))
        else:
            h = _handle
        self._h = h
        _live.add(self)
        self.device = device
        self._refresh()

    def adapt(self, flags, reuse: bool = True):
        """New geometry after refining (+1) / coarsening (-1) leaf blocks
        (one flag per leaf block, canonical order); returns (geometry,
        stats [blocks kept, blocks set up, records kept, records computed])."""
        f = np.ascontiguousarray(flags, dtype=np.int8)
        assert f.size == self.n_leaf_blocks, (f.size, self.n_leaf_blocks)
        h = _vp()
        stats = np.zeros(4, dtype=np.int64)
        _check(lib().octmg_geom_adapt(self._h, f.ctypes.data, int(reuse), C.byref(h), _ptr(stats, C.c_int64)))
        out = Geometry(self.geom, self.device, _handle=h, ctx=self.ctx)
        out._parent_desc = self.desc  # the adapted geometry calls the same level-set callback
        return out, stats

    def solve_noalloc(self, rhs, phi, iface_vals=None, domain_vals=None, rtol: float = 1e-10, max_cycles: int = 40,
                      kind: int = CYCLE_V, stream=None, raise_on_fail: bool = True) -> SolveReport:
        """One FP64 solve from phi = 0 with no device allocation
        (octmg_solve_noalloc): rhs, phi and the boundary values are float64
        device tensors; phi receives the solution."""
        for t in (rhs, phi, iface_vals, domain_vals):
            if t is not None and not (hasattr(t, "data_ptr") and t.is_cuda and str(t.dtype) == "torch.float64"
                                      and t.is_contiguous()):
                raise ValueError("solve_noalloc takes contiguous float64 device tensors")
        if rhs.numel() != self.n_leaf or phi.numel() != self.n_leaf:
            raise ValueError("rhs and phi need n_leaf values")
        if iface_vals is not None and iface_vals.numel() != self.n_iface:
            raise ValueError("iface_vals needs n_iface values")
        if domain_vals is not None and domain_vals.numel() != self.n_domain:
            raise ValueError("domain_vals needs n_domain values")
        o = SolveOpts()
        o.cycle_kind, o.max_cycles, o.zero_start, o.rtol, o.graph_mode = kind, max_cycles, 1, rtol, 0
        rep = SolveReport()
        per = {"status": np.zeros(1, dtype=np.int32), "cycles": np.zeros(1, dtype=np.int32), "r0": np.zeros(1),
               "r_final": np.zeros(1)}
        rep.rhs_status, rep.rhs_cycles = _ptr(per["status"], C.c_int), _ptr(per["cycles"], C.c_int)
        rep.rhs_r0, rep.rhs_r_final = _ptr(per["r0"], C.c_double), _ptr(per["r_final"], C.c_double)
        ptr = lambda t: None if t is None else t.data_ptr()
        st = lib().octmg_solve_noalloc(self._h, ptr(rhs), ptr(iface_vals), ptr(domain_vals), ptr(phi), C.byref(o),
                                       _stream_ptr(stream), C.byref(rep))
        rep.per_rhs = per
        if raise_on_fail:
            _check(st)
        return rep

    def leaf_blocks(self):
        """(level, x, y, z) of every leaf block in canonical order."""
        out = []
        for il in range(self.n_levels):
            pos, leaf = self.block_positions(il)
            out.extend((il, *p) for p, lf in zip(pos, leaf) if lf)
        return np.array(out, dtype=np.int64).reshape(-1, 4)

    def _refresh(self):
        info = np.zeros(8, dtype=np.int64)
        _check(lib().octmg_geom_info(self._h, _ptr(info, C.c_int64)))
        (self.n_levels, self.n_leaf, self.n_iface, self.n_domain, self.n_records, self.device_bytes,
         self.n_blocks, self.n_iface_blocks) = (int(v) for v in info)
        self.n_leaf_blocks = sum(self.level_info(il)["nleaf"] for il in range(self.n_levels))

    def close(self):
        if getattr(self, "_h", None):
            lib().octmg_geom_destroy(self._h)
            self._h = None

    def __del__(self):
        if not _finalizing():
            self.close()

    def level_info(self, level: int) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(lib().octmg_geom_level_info(self._h, level, _ptr(out, C.c_int64)))
        keys = ["n", "Nb", "nblocks", "nleaf", "nrec", "npts", "nface", "n_iface_blocks"]
        return dict(zip(keys, (int(v) for v in out)))

    def leaf_coords(self):
        xyz = np.zeros((self.n_leaf, 3))
        lvl = np.zeros(self.n_leaf, dtype=np.int32)
        _check(lib().octmg_geom_leaf_coords(self._h, _ptr(xyz, C.c_double), _ptr(lvl, C.c_int)))
        return xyz, lvl

    def iface_points(self):
        xyz = np.zeros((self.n_iface, 3))
        if self.n_iface:
            _check(lib().octmg_geom_iface_points(self._h, _ptr(xyz, C.c_double)))
        return xyz

    def domain_points(self):
        xyz = np.zeros((self.n_domain, 3))
        _check(lib().octmg_geom_domain_points(self._h, _ptr(xyz, C.c_double)))
        return xyz

    def records(self, level: int):
        n = self.level_info(level)["nrec"]
        ids = np.zeros((n, 3), dtype=np.int32)
        d = np.zeros((n, 6))
        coef = np.zeros((n, 8))
        if n:
            _check(lib().octmg_geom_records(self._h, level, _ptr(ids, C.c_int), _ptr(d, C.c_double),
                                            _ptr(coef, C.c_double)))
        return ids, d, coef

    def block_positions(self, level: int):
        nb = self.level_info(level)["nblocks"]
        pos = np.zeros((nb, 3), dtype=np.int32)
        leaf = np.zeros(nb, dtype=np.int32)
        _check(lib().octmg_geom_block_positions(self._h, level, _ptr(pos, C.c_int), _ptr(leaf, C.c_int)))
        return pos, leaf


class State:
    """Fields of n_rhs right-hand sides on a Geometry (FP64 or MIXED)."""

    def __init__(self, geometry: Geometry, n_rhs: int = 1, precision: int = FP64):
        self.geometry = geometry
        self.n_rhs = n_rhs
        self.precision = precision
        h = _vp()
        _check(lib().octmg_state_create(geometry._h, n_rhs, precision, C.byref(h)))
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            lib().octmg_state_destroy(self._h)
            self._h = None

    def __del__(self):
        if not _finalizing():
            self.close()

    def set_smoothing(self, n_down: int, n_up: int):
        _check(lib().octmg_state_set_smoothing(self._h, n_down, n_up))

    def set_launch(self, block_order=0, bottom_kind=0, bottom_max_blocks=0, graph_mode=0, pair_max_blocks=1 << 30,
                   prolong_fused=1, red_preset=1, update_fused=1):
        c = LaunchConfig(block_order, bottom_kind, bottom_max_blocks, graph_mode, pair_max_blocks, prolong_fused,
                         red_preset, update_fused)
        _check(lib().octmg_state_set_launch(self._h, C.byref(c)))

    def get_launch(self) -> dict:
        c = LaunchConfig()
        _check(lib().octmg_state_get_launch(self._h, C.byref(c)))
        return c.as_dict()

    def autotune(self, rtol: float = 1e-10, max_cycles: int = 40, kind: int = CYCLE_V, reps: int = 2, stream=None):
        """Time every candidate launch configuration; keep and return the
        fastest, with the per-candidate mean ms per solve.  The whole-solve
        graph candidates capture max_cycles cycles."""
        o = SolveOpts()
        o.cycle_kind, o.max_cycles, o.zero_start, o.rtol = kind, max_cycles, 1, rtol
        best = LaunchConfig()
        ms = np.zeros(16)
        n = C.c_int()
        _check(lib().octmg_autotune(self._h, C.byref(o), reps, _stream_ptr(stream), C.byref(best),
                                    _ptr(ms, C.c_double), C.byref(n)))
        return best.as_dict(), ms[:n.value].tolist()  # no timings on a tune-cache hit

    def set_fused_levels(self, max_blocks: int):
        """Run levels with <= max_blocks blocks in one fused launch (0: off)."""
        _check(lib().octmg_state_set_fused_levels(self._h, max_blocks))

    def _arr(self, a, n):
        """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
        if hasattr(a, "data_ptr"):
            assert a.dtype.__str__() == "torch.float64" and a.is_contiguous() and a.numel() == n
            return a.data_ptr(), int(a.is_cuda), a
        arr = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        assert arr.size == n, (arr.size, n)
        return arr.ctypes.data, 0, arr

    def set_boundary(self, iface_vals=None, domain_vals=None, stream=None):
        g = self.geometry
        pi, od1, k1 = self._arr(iface_vals, g.n_iface) if iface_vals is not None and g.n_iface else (None, 0, None)
        pd, od2, k2 = self._arr(domain_vals, g.n_domain) if domain_vals is not None else (None, 0, None)
        on_dev = od1 or od2
        _check(lib().octmg_set_boundary(self._h, pi, pd, on_dev, _stream_ptr(stream)))

    def set_boundary_fn(self, iface_fn, domain_fn, stream=None):
        g = self.geometry
        p = g.iface_points()
        q = g.domain_points()
        self.set_boundary(iface_fn(p) if len(p) else None, domain_fn(q), stream)

    def _typed(self, a, n):
        """(pointer, dtype code, on_device, keepalive) for float64 or float32
        numpy arrays and torch tensors; other host arrays become float64."""
        if hasattr(a, "data_ptr"):
            dt = str(a.dtype)
            assert dt in ("torch.float64", "torch.float32") and a.is_contiguous() and a.numel() == n, (dt, a.numel())
            return a.data_ptr(), DTYPE_F32 if dt == "torch.float32" else DTYPE_F64, int(a.is_cuda), a
        a = np.asarray(a)
        arr = np.ascontiguousarray(a, dtype=np.float32 if a.dtype == np.float32 else np.float64).reshape(-1)
        assert arr.size == n, (arr.size, n)
        return arr.ctypes.data, DTYPE_F32 if arr.dtype == np.float32 else DTYPE_F64, 0, arr

    def set_rhs(self, g, stream=None):
        p, dt, od, keep = self._typed(g, self.geometry.n_leaf * self.n_rhs)
        _check(lib().octmg_set_rhs(self._h, p, dt, od, _stream_ptr(stream)))

    def remap_from(self, other: "State", stream=None):
        """phi carried over from a state of the geometry this one was adapted from."""
        _check(lib().octmg_state_remap(other._h, self._h, _stream_ptr(stream)))

    def set_solution(self, phi, stream=None):
        p, dt, od, keep = self._typed(phi, self.geometry.n_leaf * self.n_rhs)
        _check(lib().octmg_set_solution(self._h, p, dt, od, _stream_ptr(stream)))

    def get_solution(self, out=None, stream=None, dtype=np.float64) -> np.ndarray:
        """Leaf values of phi; into `out` (a float64/float32 numpy array or
        tensor) if given, else a new host array of `dtype`."""
        n = self.geometry.n_leaf * self.n_rhs
        if out is not None:
            p, dt, od, keep = self._typed(out, n)
            if not od and keep is not out and keep.base is not out:
                raise ValueError("out must be a contiguous float64 or float32 array")
            _check(lib().octmg_get_solution(self._h, p, dt, od, _stream_ptr(stream)))
            return out
        a = np.zeros(n, dtype=np.float32 if np.dtype(dtype) == np.float32 else np.float64)
        _check(lib().octmg_get_solution(self._h, a.ctypes.data, DTYPE_F32 if a.dtype == np.float32 else DTYPE_F64, 0,
                                        _stream_ptr(stream)))
        return a.reshape(self.n_rhs, -1) if self.n_rhs > 1 else a

    def zero_solution(self, stream=None):
        _check(lib().octmg_zero_solution(self._h, _stream_ptr(stream)))

    def cycle(self, kind: int = CYCLE_V, have_guess: bool = True, stream=None):
        _check(lib().octmg_cycle(self._h, kind, int(have_guess), _stream_ptr(stream)))

    def vcycle(self, stream=None):
        self.cycle(CYCLE_V, True, stream)

    def fmg(self, have_guess: bool = True, stream=None):
        self.cycle(CYCLE_FMG, have_guess, stream)

    def gradient(self, inside_zero: bool = False, stream=None) -> np.ndarray:
        """grad phi at the leaf cell centres, [n_leaf][3] (or [n_rhs][n_leaf][3])."""
        g = self.geometry
        out = np.zeros((self.n_rhs, g.n_leaf, 3))
        _check(lib().octmg_gradient(self._h, int(inside_zero), out.ctypes.data, 0, _stream_ptr(stream)))
        return out[0] if self.n_rhs == 1 else out

    def residual_norm(self, phi_zero: bool = False, stream=None) -> np.ndarray:
        out = np.zeros(self.n_rhs)
        _check(lib().octmg_residual_norm(self._h, int(phi_zero), _ptr(out, C.c_double), _stream_ptr(stream)))
        return out

    def solve(self, rtol: float = 1e-10, max_cycles: int = 40, kind: int = CYCLE_V, zero_start: bool = False,
              stream=None, raise_on_fail: bool = True, graph_mode: int = 0) -> SolveReport:
        o = SolveOpts()
        o.cycle_kind, o.max_cycles, o.zero_start, o.rtol = kind, max_cycles, int(zero_start), rtol
        o.graph_mode = graph_mode
        rep = SolveReport()
        per = {"status": np.zeros(self.n_rhs, dtype=np.int32), "cycles": np.zeros(self.n_rhs, dtype=np.int32),
               "r0": np.zeros(self.n_rhs), "r_final": np.zeros(self.n_rhs)}
        rep.rhs_status, rep.rhs_cycles = _ptr(per["status"], C.c_int), _ptr(per["cycles"], C.c_int)
        rep.rhs_r0, rep.rhs_r_final = _ptr(per["r0"], C.c_double), _ptr(per["r_final"], C.c_double)
        st = lib().octmg_solve(self._h, C.byref(o), _stream_ptr(stream), C.byref(rep))
        rep.per_rhs = per  # per right-hand side: status, cycles, r0, r_final
        if raise_on_fail:
            _check(st)
        return rep

    def profile(self, enable: bool = True):
        _check(lib().octmg_profile_enable(self._h, int(enable)))

    def profile_read(self) -> dict:
        out = np.zeros(4)
        _check(lib().octmg_profile_read(self._h, _ptr(out, C.c_double)))
        return {"finest_half_sweeps": int(out[0]), "finest_half_sweep_ms": float(out[1]),
                "smoother_cell_updates": float(out[2]), "finest_cells": int(out[3])}

    # ---- kernel-level access (parity checks)
    def get_field(self, level: int, field: int, rhs: int = 0) -> np.ndarray:
        info = self.geometry.level_info(level)
        a = np.zeros(info["nblocks"] * info["Nb"] ** self.geometry.geom.dim)
        _check(lib().octmg_debug_get_field(self._h, level, field, rhs, _ptr(a, C.c_double)))
        return a

    def set_field(self, level: int, field: int, vals, rhs: int = 0):
        a = np.ascontiguousarray(vals, dtype=np.float64)
        _check(lib().octmg_debug_set_field(self._h, level, field, rhs, _ptr(a, C.c_double)))

    def step(self, step: int, level: int, arg: int = 0, stream=None):
        _check(lib().octmg_debug_step(self._h, step, level, arg, _stream_ptr(stream)))


def _buf(a):
    """(pointer, on_device) of a float64 numpy array or device tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffers must be contiguous float64")
        return a.ctypes.data, 0
    if not a.is_contiguous() or str(a.dtype) != "torch.float64":
        raise ValueError("tensors must be contiguous float64")
    return a.data_ptr(), 1 if a.is_cuda else 0


class Server:
    """Serving engine (octmg_server_*): continuous batching of one-rhs
    solve requests over resident geometries within a device-memory budget.

    Buffers passed to submit() are kept referenced here until their result
    has been polled."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_lanes: int = 16,
                 precision: int = MIXED, max_cycles: int = 40):
        o = ServerOpts()
        o.hbm_budget_bytes, o.max_lanes, o.precision, o.max_cycles = hbm_budget_bytes, max_lanes, precision, max_cycles
        h = C.c_void_p()
        _check(lib().octmg_server_create(device, C.byref(o), C.byref(h)))
        self._h = h
        _live.add(self)
        self._geoms = []
        self._held = {}

    def add_geometry(self, geometry: "Geometry", iface_vals=None, domain_vals=None) -> int:
        iv = None if iface_vals is None else np.ascontiguousarray(iface_vals, dtype=np.float64)
        dv = None if domain_vals is None else np.ascontiguousarray(domain_vals, dtype=np.float64)
        slot = C.c_int()
        _check(lib().octmg_server_add_geometry(self._h, geometry._h, None if iv is None else iv.ctypes.data,
                                               None if dv is None else dv.ctypes.data, C.byref(slot)))
        self._geoms.append(geometry)
        return slot.value

    def submit(self, slot: int, rhs, out, rtol: float = 1e-8) -> int:
        rp, rd = _buf(rhs)
        op, od = _buf(out)
        rid = C.c_uint64()
        _check(lib().octmg_server_submit(self._h, slot, rp, rd, op, od, rtol, C.byref(rid)))
        self._held[rid.value] = (rhs, out)
        return rid.value

    def poll(self, cap: int = 256):
        buf = (Result * cap)()
        n = C.c_int()
        _check(lib().octmg_server_poll(self._h, buf, cap, C.byref(n)))
        out = []
        for i in range(n.value):
            r = buf[i]
            self._held.pop(r.id, None)
            out.append({"id": r.id, "status": r.status, "cycles": r.cycles, "r0": r.r0, "r_final": r.r_final,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done})
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().octmg_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().octmg_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        if not _finalizing():
            try:
                self.close()
            except Exception:
                pass
