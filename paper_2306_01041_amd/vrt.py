"""ctypes binding of ``libvrt.so`` (declared in ``include/vrt.h``).

Argument marshalling only: every computation runs in the library's HIP
kernels. Host arrays are numpy; device arrays are torch tensors on the
context's GPU (used for memory and streams, never for arithmetic here). The
functions keep the C names; small classes own the context and grid handles.

Importing this module fails loudly when the library has not been built.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvrt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_01041_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

VRT_OK = 0
VRT_W_NOT_CONVERGED = 1
VRT_E_ARG = -1
VRT_E_GRID = -2
VRT_E_DAG = -3
VRT_E_HIP = -4
VRT_E_NOMEM = -5
VRT_E_NUMERIC = -6
VRT_E_STATE = -7
VRT_E_TIMEOUT = -8

VRT_TUNE_RECORD_ORDER = 1
VRT_TUNE_XCD_CHUNKS = 2
VRT_TUNE_SPIN_CAP = 3
VRT_TUNE_PERSIST_BLOCKS = 4
VRT_TUNE_RAY_AFFINITY = 5
VRT_TUNE_CHAINS = 6
VRT_TUNE_LANE_BYTES = 8
VRT_TUNE_RAY_GROUPS = 9
VRT_TUNE_INTERLEAVE = 10
VRT_TUNE_SEGMENT = 11
VRT_TUNE_REVERSE_PERSISTENT = 13
VRT_TUNE_PIPELINE = 14
VRT_TUNE_REGULAR_TILE = 15
VRT_TUNE_SHARED_LEVELS = 16

VRT_F64 = 0
VRT_F32 = 1
VRT_EXEC_PLAIN = 0
VRT_EXEC_BATCHED = 1
VRT_EXEC_GRAPH = 2
VRT_EXEC_PERSISTENT = 3
VRT_EXEC_AUTO = 4  # the launch mode the autotuner chose for the grid

_vp = ctypes.c_void_p
_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i8 = ctypes.POINTER(ctypes.c_int8)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_st = ctypes.c_int32


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


vrt_version = _sig("vrt_version", ctypes.c_char_p, [])
vrt_status_string = _sig("vrt_status_string", ctypes.c_char_p, [_st])
vrt_validate_voronoi = _sig("vrt_validate_voronoi", _st, [ctypes.c_int64, _d, _i64, _i32, _i8, _u8, _d, _d,
                                                          ctypes.c_uint32, ctypes.c_char_p, ctypes.c_int64])
vrt_ctx_create = _sig("vrt_ctx_create", _st, [ctypes.c_int32, _vp, ctypes.POINTER(_vp)])
vrt_ctx_destroy = _sig("vrt_ctx_destroy", None, [_vp])
vrt_ctx_last_error = _sig("vrt_ctx_last_error", ctypes.c_char_p, [_vp])
vrt_ctx_set_stream = _sig("vrt_ctx_set_stream", _st, [_vp, _vp])
vrt_ctx_synchronize = _sig("vrt_ctx_synchronize", _st, [_vp])
vrt_ctx_set_profiling = _sig("vrt_ctx_set_profiling", _st, [_vp, ctypes.c_int32])
vrt_ctx_profile = _sig("vrt_ctx_profile", _st, [_vp, ctypes.c_int32, _d, _i64, _i64])
vrt_ctx_profile_reset = _sig("vrt_ctx_profile_reset", _st, [_vp])
vrt_grid_create_voronoi = _sig("vrt_grid_create_voronoi", _st, [_vp, ctypes.c_int64, _d, _i64, _i32, _i8, _u8, _d,
                                                                _d, ctypes.c_uint32, ctypes.POINTER(_vp)])
vrt_grid_create_regular = _sig("vrt_grid_create_regular", _st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                                ctypes.c_double, ctypes.c_double, _d,
                                                                ctypes.POINTER(_vp)])
vrt_grid_destroy = _sig("vrt_grid_destroy", None, [_vp])
vrt_grid_set_rays = _sig("vrt_grid_set_rays", _st, [_vp, ctypes.c_int32, _d, _d, ctypes.c_double])
vrt_grid_tune = _sig("vrt_grid_tune", _st, [_vp, ctypes.c_int32, ctypes.c_int64])
vrt_grid_autotune = _sig("vrt_grid_autotune", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp,
                                                    _vp, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int64])
vrt_grid_info = _sig("vrt_grid_info", _st, [_vp, _i64, _i32, _i32, _i64])
vrt_grid_schedule = _sig("vrt_grid_schedule", _st, [_vp, ctypes.c_int32, _i32, _i32, _d, _d, _d, _i32, _i32, _i32,
                                                    _i32])
vrt_lte_continuum = _sig("vrt_lte_continuum", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _d, ctypes.c_double, _vp,
                                                    _vp, _vp, _vp])
vrt_lte_continuum_ld = _sig("vrt_lte_continuum_ld", _st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _d,
                                                          ctypes.c_double, _vp, _vp, _vp, _vp])
vrt_formal_solution = _sig("vrt_formal_solution", _st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                                        _vp, _vp, _vp, _vp])
vrt_formal_solution_ld = _sig("vrt_formal_solution_ld", _st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                              ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp])
vrt_formal_solution_noalloc = _sig("vrt_formal_solution_noalloc", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp,
                                                                        _vp, _vp, _vp, _vp])
vrt_two_level_solve = _sig("vrt_two_level_solve", _st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _d, _vp,
                                                        _vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                                        ctypes.c_double, ctypes.c_int32, _vp, _d, _i32])
vrt_two_level_solve_batched = _sig("vrt_two_level_solve_batched", _st,
                                   [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _d, _vp, _vp, _vp, _vp,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp,
                                    ctypes.c_int32, _i64, _d, _i32])
vrt_formal_solution_vjp = _sig("vrt_formal_solution_vjp", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                                                _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                                                ctypes.c_int32, ctypes.c_int32])
vrt_grid_solution_id = _sig("vrt_grid_solution_id", _st, [_vp, ctypes.POINTER(ctypes.c_int64)])
vrt_formal_solution_vjp_last = _sig("vrt_formal_solution_vjp_last", _st,
                                    [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     _vp, _vp, ctypes.c_int32, ctypes.c_int64])
vrt_formal_solution_vjp_scratch = _sig("vrt_formal_solution_vjp_scratch", _st,
                                       [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)])
vrt_emergent_scatter = _sig("vrt_emergent_scatter", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp])
vrt_lte_continuum_vjp = _sig("vrt_lte_continuum_vjp", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _d, ctypes.c_double,
                                                            _vp, _vp, _vp, _vp, _vp, _vp, _vp])
vrt_grid_device_status = _sig("vrt_grid_device_status", _st, [_vp])
vrt_grid_emergent_index = _sig("vrt_grid_emergent_index", _st, [_vp, _i64, _i32])
vrt_emergent_gather = _sig("vrt_emergent_gather", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp])
vrt_idw_map = _sig("vrt_idw_map", _st, [_vp, _vp, ctypes.c_double, _vp, _vp, _vp])
vrt_idw_apply = _sig("vrt_idw_apply", _st, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp])
vrt_synthesis_vertical = _sig("vrt_synthesis_vertical", _st, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                                              _vp, _vp, _vp, _vp, _vp, _vp])
vrt_lc_vertical = _sig("vrt_lc_vertical", _st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp])

EXPORTED = [n for n in dir() if n.startswith("vrt_")]


class VrtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{vrt_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _dev(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _prec_of(t):
    import torch

    if t.dtype == torch.float64:
        return VRT_F64
    if t.dtype == torch.float32:
        return VRT_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def validate_voronoi(n, xyz, nbr_ptr, nbr_idx, nbr_shift, wall, lo, hi, periodic_xy=True):
    """Host-only geometry check; returns (status, message)."""
    buf = ctypes.create_string_buffer(512)
    keep = [None if a is None else np.ascontiguousarray(a, dt) for a, dt in
            ((xyz, np.float64), (nbr_ptr, np.int64), (nbr_idx, np.int32), (nbr_shift, np.int8), (wall, np.uint8),
             (lo, np.float64), (hi, np.float64))]
    ptrs = [None if a is None else _p(a, t) for a, t in zip(keep, (_d, _i64, _i32, _i8, _u8, _d, _d))]
    st = vrt_validate_voronoi(int(n), *ptrs, 1 if periodic_xy else 0, buf, 512)
    return st, buf.value.decode()


# Live contexts, closed (with their grids) by an exit hook while the HIP runtime
# and torch's streams still exist. Garbage collection during interpreter
# shutdown runs in no defined order relative to the runtime's own teardown, so
# __del__ makes no library call once the interpreter is finalizing.
_live_contexts = weakref.WeakSet()


def _close_all_contexts():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


atexit.register(_close_all_contexts)


class Context:
    """A library context on one GPU, enqueuing on a HIP stream (default: torch's current stream).

    Close it with close() (or let the exit hook do it); a context that is
    garbage-collected while the interpreter runs is closed then."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream_obj = stream
        h = _vp()
        st = vrt_ctx_create(int(device), _vp(stream.cuda_stream), ctypes.byref(h))
        if st != VRT_OK:
            raise VrtError(st, "vrt_ctx_create failed")
        self.handle = h
        self.device = device
        _live_contexts.add(self)

    def check(self, st):
        if st < 0:
            raise VrtError(st, vrt_ctx_last_error(self.handle).decode())
        return st

    def set_stream(self, stream):
        self._stream_obj = stream
        self.check(vrt_ctx_set_stream(self.handle, _vp(stream.cuda_stream)))

    def synchronize(self):
        self.check(vrt_ctx_synchronize(self.handle))

    def set_profiling(self, on: bool):
        self.check(vrt_ctx_set_profiling(self.handle, 1 if on else 0))

    def profile(self, kernel: int):
        """(ms, launches, units) summed over instrumented launches of a kernel class."""
        ms = ctypes.c_double()
        nl = ctypes.c_int64()
        un = ctypes.c_int64()
        self.check(vrt_ctx_profile(self.handle, int(kernel), ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(un)))
        return ms.value, nl.value, un.value

    def profile_reset(self):
        self.check(vrt_ctx_profile_reset(self.handle))

    def close(self):
        if self.handle:
            vrt_ctx_destroy(self.handle)
            self.handle = None
        _live_contexts.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone at exit)
        if _finalizing() or not self.handle:
            return
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """A Voronoi or regular grid handle with its quadrature and schedules."""

    def __init__(self, ctx: Context, handle, kind: str):
        self.ctx = ctx
        self.handle = handle
        self.kind = kind

    @classmethod
    def voronoi(cls, ctx: Context, xyz, nbr_ptr, nbr_idx, nbr_shift, wall, lo, hi, periodic_xy=True):
        xyz = np.ascontiguousarray(xyz, np.float64)
        ptr = np.ascontiguousarray(nbr_ptr, np.int64)
        idx = np.ascontiguousarray(nbr_idx, np.int32)
        sh = None if nbr_shift is None else np.ascontiguousarray(nbr_shift, np.int8)
        wall = np.ascontiguousarray(wall, np.uint8)
        lo = np.ascontiguousarray(lo, np.float64)
        hi = np.ascontiguousarray(hi, np.float64)
        h = _vp()
        ctx.check(vrt_grid_create_voronoi(ctx.handle, xyz.shape[0], _p(xyz, _d), _p(ptr, _i64), _p(idx, _i32),
                                          _p(sh, _i8), _p(wall, _u8), _p(lo, _d), _p(hi, _d),
                                          1 if periodic_xy else 0, ctypes.byref(h)))
        return cls(ctx, h, "voronoi")

    @classmethod
    def from_synth(cls, ctx: Context, g):
        return cls.voronoi(ctx, g.xyz, g.nbr_ptr, g.nbr_idx, g.nbr_shift, g.wall, g.lo, g.hi, g.periodic_xy)

    @classmethod
    def regular(cls, ctx: Context, nx, ny, z, dx, dy):
        z = np.ascontiguousarray(z, np.float64)
        h = _vp()
        ctx.check(vrt_grid_create_regular(ctx.handle, int(nx), int(ny), len(z), float(dx), float(dy), _p(z, _d),
                                          ctypes.byref(h)))
        g = cls(ctx, h, "regular")
        g.z = z.copy()
        return g

    def set_rays(self, dirs, w, r_exp: float = 7.0):
        dirs = np.ascontiguousarray(dirs, np.float64)
        w = np.ascontiguousarray(w, np.float64)
        self.ctx.check(vrt_grid_set_rays(self.handle, dirs.shape[0], _p(dirs, _d), _p(w, _d), float(r_exp)))

    def tune(self, knob: int, value: int):
        self.ctx.check(vrt_grid_tune(self.handle, int(knob), int(value)))

    def info(self):
        n = ctypes.c_int64()
        r = ctypes.c_int32()
        L = ctypes.c_int32()
        fb = ctypes.c_int64()
        self.ctx.check(vrt_grid_info(self.handle, ctypes.byref(n), ctypes.byref(r), ctypes.byref(L), ctypes.byref(fb)))
        return dict(n_sites=n.value, n_rays=r.value, max_levels=L.value, n_fallback=fb.value)

    def schedule(self, ray: int):
        n = self.info()["n_sites"]
        k1 = np.empty(n, np.int32)
        k2 = np.empty(n, np.int32)
        w1 = np.empty(n, np.float64)
        d1 = np.empty(n, np.float64)
        d2 = np.empty(n, np.float64)
        lev = np.empty(n, np.int32)
        order = np.empty(n, np.int32)
        lp = np.empty(n + 1, np.int32)
        nl = ctypes.c_int32()
        self.ctx.check(vrt_grid_schedule(self.handle, int(ray), _p(k1, _i32), _p(k2, _i32), _p(w1, _d), _p(d1, _d),
                                         _p(d2, _d), _p(lev, _i32), _p(order, _i32), _p(lp, _i32), ctypes.byref(nl)))
        return dict(k1=k1, k2=k2, w1=w1, ds1=d1, ds2=d2, level=lev, order=order, level_ptr=lp[: nl.value + 1].copy(),
                    n_levels=nl.value)

    def solution_id(self) -> int:
        """Identifier of the grid's last solution (see formal_solution_vjp_last)."""
        out = ctypes.c_int64(0)
        self.ctx.check(vrt_grid_solution_id(self.handle, ctypes.byref(out)))
        return int(out.value)

    def device_status(self):
        """Synchronise and raise VrtError(VRT_E_TIMEOUT) if a bounded device wait gave up."""
        self.ctx.check(vrt_grid_device_status(self.handle))

    def emergent_index(self):
        R = self.info()["n_rays"]
        off = np.empty(R + 1, np.int64)
        self.ctx.check(vrt_grid_emergent_index(self.handle, _p(off, _i64), None))
        sites = np.empty(int(off[-1]), np.int32)
        self.ctx.check(vrt_grid_emergent_index(self.handle, _p(off, _i64), _p(sites, _i32)))
        return off, sites

    def close(self):
        # a destroyed context has already freed its grids
        if self.handle and self.ctx.handle:
            vrt_grid_destroy(self.handle)
        self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing() or not self.handle:
            return
        try:
            self.close()
        except Exception:
            pass


def _need(t, shape, dtype, name):
    """Host-side guard: a device tensor of exactly this shape and dtype, contiguous, on a GPU."""
    if t is None:
        return
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def row_stride(tensors, shape, dtype):
    """The common row stride (elements) of [n, nl] tensors whose rows are
    unit-stride and do not overlap (None entries are skipped): views such as
    cs[:, 0] and cs[:, 1] of one [n, 2, nl] array, whose rows lie 2 nl apart.
    Raises ValueError for another shape or dtype, a non-unit element stride,
    overlapping rows or strides that differ between the tensors."""
    n, nl = shape
    ld = None
    for t, name in tensors:
        if t is None:
            continue
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if t.dtype != dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
        if nl > 1 and t.stride(1) != 1:
            raise ValueError(f"{name}: the entries of a row must be adjacent")
        r = t.stride(0) if n > 1 else nl
        if r < nl:
            raise ValueError(f"{name}: rows {r} apart overlap rows of {nl} entries")
        if ld is not None and r != ld:
            raise ValueError(f"{name}: rows {r} apart, the other inputs' rows {ld} apart")
        ld = r
    return nl if ld is None else ld


def _rows_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def lte_continuum(grid: Grid, lam, kappa0, T, rho, chi, S):
    """chi = kappa0 rho^2 T^9, S = B_lambda(T) into device tensors chi, S [n, nl]
    (their dtype sets the precision). chi and S may be row-strided views with a
    common row stride, e.g. cs[:, 0] and cs[:, 1] of one [n, 2, nl] array."""
    import torch

    lam = np.ascontiguousarray(np.atleast_1d(lam), np.float64)
    n = grid.info()["n_sites"]
    _need(T, (n,), torch.float64, "T")
    _need(rho, (n,), torch.float64, "rho")
    ld = row_stride(((chi, "chi"), (S, "S")), (n, len(lam)), chi.dtype)
    grid.ctx.check(vrt_lte_continuum_ld(grid.handle, _prec_of(chi), len(lam), int(ld), _p(lam, _d), float(kappa0),
                                        _dev(T), _dev(rho), _rows_ptr(chi), _rows_ptr(S)))


def formal_solution(grid: Grid, chi, S, J, I_bottom=None, I_top=None, I_rays=None, exec_mode=VRT_EXEC_BATCHED):
    """Formal solution of every ray and J (device tensors [n, nl]; I_rays [R, n,
    nl] optional). The inputs chi, S, I_bottom and I_top may be row-strided views
    with one common row stride (vrt_formal_solution_ld), e.g. chi = cs[:, 0] and
    S = cs[:, 1] of one [n, 2, nl] array; J and I_rays are contiguous."""
    inf = grid.info()
    n, R = inf["n_sites"], inf["n_rays"]
    if chi.dim() != 2:
        raise ValueError("chi must be [n_sites, n_lambda]")
    nl = chi.shape[1]
    ld = row_stride(((chi, "chi"), (S, "S"), (I_bottom, "I_bottom"), (I_top, "I_top")), (n, nl), chi.dtype)
    _need(J, (n, nl), chi.dtype, "J")
    _need(I_rays, (R, n, nl), chi.dtype, "I_rays")
    if ld == nl:
        grid.ctx.check(vrt_formal_solution(grid.handle, _prec_of(chi), int(exec_mode), int(nl), _rows_ptr(chi),
                                           _rows_ptr(S), _rows_ptr(I_bottom), _rows_ptr(I_top), _dev(J),
                                           _dev(I_rays)))
    else:
        grid.ctx.check(vrt_formal_solution_ld(grid.handle, _prec_of(chi), int(exec_mode), int(nl), int(ld),
                                              _rows_ptr(chi), _rows_ptr(S), _rows_ptr(I_bottom), _rows_ptr(I_top),
                                              _dev(J), _dev(I_rays)))


def formal_solution_noalloc(grid: Grid, chi, S, J, I_bottom=None, I_top=None):
    """vrt_formal_solution_noalloc: the batched formal solution with the per-ray
    intensities in the library's static per-GPU buffer (no allocation; calls on
    one GPU must not overlap)."""
    inf = grid.info()
    n = inf["n_sites"]
    if chi.dim() != 2:
        raise ValueError("chi must be [n_sites, n_lambda]")
    nl = chi.shape[1]
    for t, name in ((chi, "chi"), (S, "S"), (J, "J"), (I_bottom, "I_bottom"), (I_top, "I_top")):
        _need(t, (n, nl), chi.dtype, name)
    grid.ctx.check(vrt_formal_solution_noalloc(grid.handle, _prec_of(chi), int(nl), _dev(chi), _dev(S),
                                               _dev(I_bottom), _dev(I_top), _dev(J)))


def emergent_gather(grid: Grid, out, I_rays=None):
    """Emergent intensities of the last formal solution into out [total, nl] (see Grid.emergent_index)."""
    inf = grid.info()
    off, _ = grid.emergent_index()
    if out.dim() != 2:
        raise ValueError("out must be [n_emergent, n_lambda]")
    nl = out.shape[1]
    _need(out, (int(off[-1]), nl), out.dtype, "out")
    _need(I_rays, (inf["n_rays"], inf["n_sites"], nl), out.dtype, "I_rays")
    grid.ctx.check(vrt_emergent_gather(grid.handle, _prec_of(out), int(nl), _dev(I_rays), _dev(out)))


def autotune(grid: Grid, chi, S, J, I_bottom=None, I_top=None, I_rays=None, reps: int = 5):
    """Time the grid's launch/layout knobs on this formal solution, keep the fastest; returns the report dict."""
    import json

    inf = grid.info()
    n, R = inf["n_sites"], inf["n_rays"]
    nl = chi.shape[1]
    for t, name in ((chi, "chi"), (S, "S"), (J, "J"), (I_bottom, "I_bottom"), (I_top, "I_top")):
        _need(t, (n, nl), chi.dtype, name)
    _need(I_rays, (R, n, nl), chi.dtype, "I_rays")
    buf = ctypes.create_string_buffer(16384)
    grid.ctx.check(vrt_grid_autotune(grid.handle, _prec_of(chi), int(nl), _dev(chi), _dev(S), _dev(I_bottom),
                                     _dev(I_top), _dev(J), _dev(I_rays), int(reps), buf, 16384))
    return json.loads(buf.value.decode() or "{}")


def two_level_solve(grid: Grid, wlam, phi, chi_line, chi_cont, B, eps, S_line, max_iter=1000, tol=1e-3,
                    sweep_dtype=None, exec_mode=VRT_EXEC_GRAPH, accel=False):
    """Lambda iteration of the two-level line; S_line (device float64 [n]) is updated in place.

    Returns (status, n_iter, dS history as numpy). status is VRT_OK or VRT_W_NOT_CONVERGED.
    """
    import torch

    sweep_dtype = torch.float32 if sweep_dtype is None else sweep_dtype
    inf = grid.info()
    n = inf["n_sites"]
    wlam = np.ascontiguousarray(wlam, np.float64)
    nl = len(wlam)
    _need(phi, (n, nl), torch.float64, "phi")
    for t, name in ((chi_line, "chi_line"), (chi_cont, "chi_cont"), (B, "B"), (S_line, "S_line")):
        _need(t, (n,), torch.float64, name)
    hist = np.zeros(max(int(max_iter), 1), np.float64)
    it = ctypes.c_int32()
    prec = VRT_F32 if sweep_dtype == torch.float32 else VRT_F64
    st = grid.ctx.check(vrt_two_level_solve(grid.handle, prec, int(exec_mode), nl, _p(wlam, _d), _dev(phi),
                                            _dev(chi_line), _dev(chi_cont), _dev(B), float(eps), int(max_iter),
                                            float(tol), 1 if accel else 0, _dev(S_line), _p(hist, _d),
                                            ctypes.byref(it)))
    return st, it.value, hist[: it.value].copy()


def two_level_solve_batched(grid: Grid, atm_ptr, wlam, phi, chi_line, chi_cont, B, eps, S_line, max_iter=1000,
                            tol=1e-3, sweep_dtype=None, exec_mode=VRT_EXEC_GRAPH, accel=False):
    """Lambda iteration of independent atmospheres stored as one grid (atmosphere a owns
    sites atm_ptr[a]:atm_ptr[a+1]); each converges and freezes on its own.

    Returns (status, n_iter per atmosphere, dS history [iterations, n_atm] with -1 after
    an atmosphere stopped).
    """
    import torch

    sweep_dtype = torch.float32 if sweep_dtype is None else sweep_dtype
    n = grid.info()["n_sites"]
    ptr = np.ascontiguousarray(atm_ptr, np.int64)
    n_atm = len(ptr) - 1
    if n_atm < 1:
        raise ValueError("atm_ptr needs at least two entries")
    wlam = np.ascontiguousarray(wlam, np.float64)
    nl = len(wlam)
    _need(phi, (n, nl), torch.float64, "phi")
    for t, name in ((chi_line, "chi_line"), (chi_cont, "chi_cont"), (B, "B"), (S_line, "S_line")):
        _need(t, (n,), torch.float64, name)
    hist = np.zeros((max(int(max_iter), 1), n_atm), np.float64)
    its = np.zeros(n_atm, np.int32)
    prec = VRT_F32 if sweep_dtype == torch.float32 else VRT_F64
    st = grid.ctx.check(vrt_two_level_solve_batched(grid.handle, prec, int(exec_mode), nl, _p(wlam, _d), _dev(phi),
                                                    _dev(chi_line), _dev(chi_cont), _dev(B), float(eps),
                                                    int(max_iter), float(tol), 1 if accel else 0, _dev(S_line),
                                                    n_atm, _p(ptr, _i64), _p(hist, _d), _p(its, _i32)))
    return st, its, hist[: int(its.max(initial=0))].copy()


def formal_solution_vjp(grid: Grid, chi, S, dL_dI=None, dL_dJ=None, I_bottom=None, I_top=None, I_rays=None,
                        ray_group: int = 0, checkpoint_levels: int = 0):
    """(dL/dchi, dL/dS, dL/dI_bottom, dL/dI_top) as new device tensors [n, nl].

    Without I_rays the forward intensities are recomputed ray group by ray
    group; checkpoint_levels = k > 0 keeps only per-level-chunk checkpoints of
    them (chunks of k level steps) and recomputes each chunk before its
    reverse steps: less memory, bit-identical results."""
    import torch

    inf = grid.info()
    n, R = inf["n_sites"], inf["n_rays"]
    nl = chi.shape[1]
    for t, name in ((chi, "chi"), (S, "S"), (dL_dJ, "dL_dJ"), (I_bottom, "I_bottom"), (I_top, "I_top")):
        _need(t, (n, nl), chi.dtype, name)
    _need(I_rays, (R, n, nl), chi.dtype, "I_rays")
    _need(dL_dI, (R, n, nl), chi.dtype, "dL_dI")
    outs = [torch.empty((n, nl), dtype=chi.dtype, device=chi.device) for _ in range(4)]
    grid.ctx.check(vrt_formal_solution_vjp(grid.handle, _prec_of(chi), int(nl), _dev(chi), _dev(S), _dev(I_bottom),
                                           _dev(I_top), _dev(I_rays), _dev(dL_dI), _dev(dL_dJ),
                                           *[_dev(o) for o in outs], int(ray_group), int(checkpoint_levels)))
    return tuple(outs)


def formal_solution_vjp_last(grid: Grid, solution_id: int, chi, S, dL_dI=None, dL_dJ=None, I_bottom=None,
                             I_top=None, ray_group: int = 0):
    """formal_solution_vjp with the forward intensities of the grid's last formal
    solution (the one whose Grid.solution_id() was `solution_id`), converted to
    chi's precision instead of recomputed. Raises VrtError (VRT_E_STATE) when
    the grid has solved again since, or that solution kept no rows of its own."""
    import torch

    inf = grid.info()
    n, R = inf["n_sites"], inf["n_rays"]
    nl = chi.shape[1]
    for t, name in ((chi, "chi"), (S, "S"), (dL_dJ, "dL_dJ"), (I_bottom, "I_bottom"), (I_top, "I_top")):
        _need(t, (n, nl), chi.dtype, name)
    _need(dL_dI, (R, n, nl), chi.dtype, "dL_dI")
    outs = [torch.empty((n, nl), dtype=chi.dtype, device=chi.device) for _ in range(4)]
    grid.ctx.check(vrt_formal_solution_vjp_last(grid.handle, _prec_of(chi), int(nl), _dev(chi), _dev(S),
                                                _dev(I_bottom), _dev(I_top), _dev(dL_dI), _dev(dL_dJ),
                                                *[_dev(o) for o in outs], int(ray_group), int(solution_id)))
    return tuple(outs)


def formal_solution_vjp_scratch(grid: Grid, dtype, n_lambda: int, keep_intensities: bool = False,
                                ray_group: int = 0, checkpoint_levels: int = 0) -> int:
    """Device bytes of scratch that formal_solution_vjp holds for these settings."""
    import torch

    out = ctypes.c_int64(0)
    grid.ctx.check(vrt_formal_solution_vjp_scratch(grid.handle, VRT_F32 if dtype == torch.float32 else VRT_F64,
                                                   int(n_lambda), 1 if keep_intensities else 0, int(ray_group),
                                                   int(checkpoint_levels), ctypes.byref(out)))
    return int(out.value)


def emergent_scatter(grid: Grid, dL_dIem, dL_dI):
    inf = grid.info()
    off, _ = grid.emergent_index()
    nl = dL_dIem.shape[1]
    _need(dL_dIem, (int(off[-1]), nl), dL_dIem.dtype, "dL_dIem")
    _need(dL_dI, (inf["n_rays"], inf["n_sites"], nl), dL_dIem.dtype, "dL_dI")
    grid.ctx.check(vrt_emergent_scatter(grid.handle, _prec_of(dL_dIem), int(nl), _dev(dL_dIem), _dev(dL_dI)))


def lte_continuum_vjp(grid: Grid, lam, kappa0, T, rho, dL_dchi, dL_dS, dL_dIbottom=None):
    """(dL/dT, dL/drho) as new float64 device tensors [n]."""
    import torch

    lam = np.ascontiguousarray(np.atleast_1d(lam), np.float64)
    n = grid.info()["n_sites"]
    _need(T, (n,), torch.float64, "T")
    _need(rho, (n,), torch.float64, "rho")
    for t, name in ((dL_dchi, "dL_dchi"), (dL_dS, "dL_dS"), (dL_dIbottom, "dL_dIbottom")):
        _need(t, (n, len(lam)), dL_dchi.dtype, name)
    gT = torch.empty((n,), dtype=torch.float64, device=T.device)
    gr = torch.empty_like(gT)
    grid.ctx.check(vrt_lte_continuum_vjp(grid.handle, _prec_of(dL_dchi), len(lam), _p(lam, _d), float(kappa0),
                                         _dev(T), _dev(rho), _dev(dL_dchi), _dev(dL_dS), _dev(dL_dIbottom),
                                         _dev(gT), _dev(gr)))
    return gT, gr


def _make_lte_emergent():
    import torch

    class LTEEmergent(torch.autograd.Function):
        """Emergent intensities of the grey LTE continuum as a differentiable
        function of per-site temperature and density (float64 [n] each).

        Forward: chi, S = lte_continuum(T, rho); formal solution; emergent
        gather. Backward: emergent scatter, the hand-written reverse sweep
        (vrt_formal_solution_vjp_last on the forward solution's own rows when
        nothing has solved on the grid since, else vrt_formal_solution_vjp,
        which recomputes them) and the LTE chain rule; every step runs in the
        library's kernels."""

        @staticmethod
        def forward(fctx, T, rho, grid, lam, kappa0, dtype, keep_intensities, ray_group, emergent_dtype,
                    checkpoint_levels):
            inf = grid.info()
            n, R = inf["n_sites"], inf["n_rays"]
            lam = np.ascontiguousarray(np.atleast_1d(lam), np.float64)
            nl = len(lam)
            dev = T.device
            fdt = dtype if emergent_dtype is None else emergent_dtype
            mixed = fdt != dtype
            # the sweep whose emergent intensities are returned (precision fdt)
            chi_f = torch.empty((n, nl), dtype=fdt, device=dev)
            S_f = torch.empty_like(chi_f)
            J = torch.empty_like(chi_f)
            I = torch.empty((R, n, nl), dtype=fdt, device=dev) if keep_intensities and not mixed else None
            lte_continuum(grid, lam, kappa0, T, rho, chi_f, S_f)
            # without rows to keep, on a Voronoi grid, the persistent sweep into
            # the library's own (sign-encoded) rows; rows kept for the backward
            # pass are fresh buffers every call, so they take eager level steps
            # (a captured graph would be rebuilt for each)
            fast = I is None and grid.kind == "voronoi"
            formal_solution(grid, chi_f, S_f, J, I_rays=I,
                            exec_mode=VRT_EXEC_PERSISTENT if fast else VRT_EXEC_BATCHED)
            # the backward pass may take this solution's rows (all rays at once)
            # instead of recomputing them, if nothing has solved on the grid
            # since; not when ray groups or checkpoints bound its memory
            reuse = I is None and checkpoint_levels == 0 and ray_group == 0
            fctx.solution = grid.solution_id() if reuse else None
            off, _ = grid.emergent_index()
            em = torch.empty((int(off[-1]), nl), dtype=fdt, device=dev)
            emergent_gather(grid, em, I_rays=I)
            if mixed:
                # the reverse sweep runs in `dtype` on fields of that precision; it
                # recomputes its own forward intensities ray group by ray group
                chi = torch.empty((n, nl), dtype=dtype, device=dev)
                S = torch.empty_like(chi)
                lte_continuum(grid, lam, kappa0, T, rho, chi, S)
            else:
                chi, S = chi_f, S_f
            fctx.grid, fctx.lam, fctx.kappa0, fctx.ray_group = grid, lam, kappa0, ray_group
            fctx.checkpoint_levels = checkpoint_levels
            fctx.I = I
            fctx.save_for_backward(T, rho, chi, S)
            return em

        @staticmethod
        def backward(fctx, g_em):
            T, rho, chi, S = fctx.saved_tensors
            grid = fctx.grid
            inf = grid.info()
            gI = torch.empty((inf["n_rays"], inf["n_sites"], chi.shape[1]), dtype=chi.dtype, device=chi.device)
            emergent_scatter(grid, g_em.contiguous().to(chi.dtype), gI)
            out = None
            if fctx.solution is not None:
                try:
                    out = formal_solution_vjp_last(grid, fctx.solution, chi, S, dL_dI=gI, ray_group=fctx.ray_group)
                except VrtError as e:
                    if e.status != VRT_E_STATE:
                        raise
                    # the grid solved again since the forward pass: recompute
            if out is None:
                out = formal_solution_vjp(grid, chi, S, dL_dI=gI, I_rays=fctx.I, ray_group=fctx.ray_group,
                                          checkpoint_levels=fctx.checkpoint_levels)
            g_chi, g_S, g_Ib, _ = out
            gT, gr = lte_continuum_vjp(grid, fctx.lam, fctx.kappa0, T, rho, g_chi, g_S, g_Ib)
            return gT, gr, None, None, None, None, None, None, None, None

    return LTEEmergent


_LTE_EMERGENT = None


def lte_emergent(T, rho, grid: Grid, lam, kappa0, dtype=None, keep_intensities=True, ray_group=0,
                 emergent_dtype=None, checkpoint_levels=0):
    """Differentiable emergent intensities [n_emergent, nl] (see LTEEmergent).

    dtype is the precision of the sweeps (float32 by default). emergent_dtype
    is the precision of the forward sweep whose intensities are returned; by
    default float64 when the sweeps are float32: a misfit's residuals are often
    a fraction of a percent of the intensities, and a single-precision forward
    sweep's ~1e-6 rounding would then reach the gradient at ~1e-4. The reverse
    sweep still runs in single precision. Pass emergent_dtype=torch.float32 for an all-single-precision
    pipeline (faster forward, gradients good to ~1e-3 of central differences
    in that regime).

    Without intensities of its own to keep (the default mixed-precision
    pipeline, or keep_intensities=False) the forward sweep runs into the
    library's rows, and the backward pass takes its forward intensities from
    those rows, rounded to the sweep precision, if nothing has solved on the
    grid in between; otherwise it recomputes them in the sweep precision.

    Memory: keep_intensities=False holds no intensity tensor between the passes
    (the backward pass takes the library's rows as above, or recomputes them),
    ray_group bounds the
    rays whose adjoint rows are held at once, and checkpoint_levels = k > 0
    keeps only per-level-chunk checkpoints of the recomputed intensities; with
    either of the last two the backward pass always recomputes.
    """
    import torch

    global _LTE_EMERGENT
    if _LTE_EMERGENT is None:
        _LTE_EMERGENT = _make_lte_emergent()
    dtype = torch.float32 if dtype is None else dtype
    if emergent_dtype is None:
        emergent_dtype = torch.float64 if dtype == torch.float32 else dtype
    return _LTE_EMERGENT.apply(T, rho, grid, lam, kappa0, dtype, keep_intensities, ray_group, emergent_dtype,
                               checkpoint_levels)


# ----------------------------------------------------------------------------
# final synthesis on the regular grid
# ----------------------------------------------------------------------------

def _pair(voronoi: Grid, regular: Grid):
    if voronoi.kind != "voronoi" or regular.kind != "regular":
        raise ValueError("expected a Voronoi grid and a regular grid")
    return voronoi.info()["n_sites"], regular.info()["n_sites"]


def idw_map(voronoi: Grid, regular: Grid, power: float = 1.0, with_d2: bool = False):
    """Two nearest Voronoi sites of every regular point and the inverse-distance
    weight of the nearer one: (idx int32 [m, 2], w1 float64 [m][, d2 [m, 2]]) on
    the GPU. Blocks."""
    import torch

    _, m = _pair(voronoi, regular)
    dev = torch.device("cuda", regular.ctx.device)
    idx = torch.empty((m, 2), dtype=torch.int32, device=dev)
    w1 = torch.empty(m, dtype=torch.float64, device=dev)
    d2 = torch.empty((m, 2), dtype=torch.float64, device=dev) if with_d2 else None
    regular.ctx.check(vrt_idw_map(voronoi.handle, regular.handle, float(power), _dev(idx), _dev(w1), _dev(d2)))
    return (idx, w1, d2) if with_d2 else (idx, w1)


def idw_apply(voronoi: Grid, regular: Grid, idx, w1, src, dst=None):
    """Interpolate src (float64 [n_sites] or [n_sites, k]) to the regular points."""
    import torch

    n, m = _pair(voronoi, regular)
    k = 1 if src.dim() == 1 else src.shape[1]
    _need(idx, (m, 2), torch.int32, "idx")
    _need(w1, (m,), torch.float64, "w1")
    _need(src, (n,) if src.dim() == 1 else (n, k), torch.float64, "src")
    shape = (m,) if src.dim() == 1 else (m, k)
    if dst is None:
        dst = torch.empty(shape, dtype=torch.float64, device=src.device)
    _need(dst, shape, torch.float64, "dst")
    regular.ctx.check(vrt_idw_apply(voronoi.handle, regular.handle, int(k), _dev(idx), _dev(w1), _dev(src),
                                    _dev(dst)))
    return dst


def synthesis_vertical(voronoi: Grid, regular: Grid, idx, w1, S_line, phi, chi_line, chi_cont, B, I_bottom=None,
                       out=None):
    """Emergent line intensity at mu = 1, [ny nx, n_lambda] in phi's dtype, from
    S_line on the Voronoi sites and the line data on the regular points."""
    import torch

    n, m = _pair(voronoi, regular)
    if phi.dim() != 2:
        raise ValueError("phi must be [n_points, n_lambda]")
    nl = phi.shape[1]
    ncol = m // len(regular.z)
    _need(idx, (m, 2), torch.int32, "idx")
    _need(w1, (m,), torch.float64, "w1")
    _need(S_line, (n,), torch.float64, "S_line")
    _need(phi, (m, nl), phi.dtype, "phi")
    for t, name in ((chi_line, "chi_line"), (chi_cont, "chi_cont"), (B, "B")):
        _need(t, (m,), torch.float64, name)
    _need(I_bottom, (ncol, nl), phi.dtype, "I_bottom")
    if out is None:
        out = torch.empty((ncol, nl), dtype=phi.dtype, device=phi.device)
    _need(out, (ncol, nl), phi.dtype, "out")
    regular.ctx.check(vrt_synthesis_vertical(voronoi.handle, regular.handle, _prec_of(phi), int(nl), _dev(idx),
                                             _dev(w1), _dev(S_line), _dev(phi), _dev(chi_line), _dev(chi_cont),
                                             _dev(B), _dev(I_bottom), _dev(out)))
    return out


def lc_vertical(regular: Grid, chi, S, I_bottom=None, out=None):
    """Intensity at the top of every column at mu = 1 for chi, S [n_points, n_lambda]."""
    m = regular.info()["n_sites"]
    if chi.dim() != 2:
        raise ValueError("chi must be [n_points, n_lambda]")
    nl = chi.shape[1]
    ncol = m // len(regular.z)
    _need(chi, (m, nl), chi.dtype, "chi")
    _need(S, (m, nl), chi.dtype, "S")
    _need(I_bottom, (ncol, nl), chi.dtype, "I_bottom")
    if out is None:
        import torch

        out = torch.empty((ncol, nl), dtype=chi.dtype, device=chi.device)
    _need(out, (ncol, nl), chi.dtype, "out")
    regular.ctx.check(vrt_lc_vertical(regular.handle, _prec_of(chi), int(nl), _dev(chi), _dev(S), _dev(I_bottom),
                                      _dev(out)))
    return out
