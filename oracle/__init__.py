"""FP64 CPU oracle for the formal solution on Voronoi and regular grids.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg, never by the product package. It
shares no code with the HIP library. The arithmetic lives in plain C
(``vrt_oracle.c``, FP64, no fused multiply-add, no fast-math) and in short
numpy routines here; the module header of the C file lists the passages of the
paper each routine follows and the readings taken where the paper is silent.

Parity status: every routine here is pinned by the ``-m "not gpu"`` tests
(closed forms, brute force, independent re-derivations); none is "parity
unpinned" except the searchlight peak, which the paper only states roughly.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vrt_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i8 = ctypes.POINTER(ctypes.c_int8)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle's C core into ``oracle/liborc.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
               "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_psi.argtypes = [ctypes.c_double, _d, _d, _d]
        L.orc_dpsi.argtypes = [ctypes.c_double, _d, _d]
        L.orc_select.argtypes = [ctypes.c_int64, _d, _i64, _i32, _i8, _u8, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, _d, ctypes.c_double, _i32, _i32, _d, _d, _d, _i64]
        L.orc_select.restype = ctypes.c_int
        L.orc_levels.argtypes = [ctypes.c_int64, _d, ctypes.c_int32, _d, _i32, _i32, _i32, _i32, _i32, _i32]
        L.orc_levels.restype = ctypes.c_int
        L.orc_height_order.argtypes = [ctypes.c_int64, _d, ctypes.c_double, _i64]
        L.orc_fs_voronoi.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _i32, _i32,
                                     _d, _d, _d, _d, _d, _d, _d, _d, _d]
        L.orc_fs_voronoi.restype = ctypes.c_int
        L.orc_fs_regular.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, _d, ctypes.c_int32, _d, _d, ctypes.c_int32, _d, _d, _d,
                                     _d, _d, _d]
        L.orc_fs_regular.restype = ctypes.c_int
        L.orc_planck.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_planck.restype = ctypes.c_double
        L.orc_dplanck_dT.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_dplanck_dT.restype = ctypes.c_double
        L.orc_lte.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, ctypes.c_double, _d, _d, _d, _d]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_fs_voronoi_vjp.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _i32, _i32,
                                         _d, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d]
        L.orc_fs_voronoi_vjp.restype = ctypes.c_int
        L.orc_lambda_diag.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _i32, _i32, _d, _d, _d,
                                      _d, _d]
        L.orc_lambda_diag.restype = None
        L.orc_lte_vjp.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, ctypes.c_double, _d, _d, _d, _d, _d, _d, _d]
        L.orc_bezier_weights.argtypes = [ctypes.c_double, _d, _d, _d, _d]
        L.orc_bezier_weights.restype = None
        L.orc_fs_voronoi_bezier.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _i32, _i32,
                                            _d, _d, _d, _i32, _i32, _d, _d, _d, _d, _d, _d, _d, _d, _d]
        L.orc_fs_voronoi_bezier.restype = ctypes.c_int
        L.orc_idw2.argtypes = [ctypes.c_int64, _d, ctypes.c_int64, _d, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, _i32, _d, _d]
        L.orc_idw2.restype = None
        L.orc_lc_vertical.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _d, _d]
        L.orc_lc_vertical.restype = None
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------------------
# segment weights
# ----------------------------------------------------------------------------

def psi(x: float):
    """(e^-x, Psi_u(x), Psi_0(x)) for S linear along a segment of optical depth x."""
    E, pu, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_psi(float(x), ctypes.byref(E), ctypes.byref(pu), ctypes.byref(p0))
    return E.value, pu.value, p0.value


def dpsi(x: float):
    """(dPsi_u/dx, dPsi_0/dx)."""
    du, d0 = ctypes.c_double(), ctypes.c_double()
    lib().orc_dpsi(float(x), ctypes.byref(du), ctypes.byref(d0))
    return du.value, d0.value


# ----------------------------------------------------------------------------
# upwind selection and levels
# ----------------------------------------------------------------------------

class Selection:
    """Per-(ray, site) upwind records: k1, k2 int32 [R, n]; w1, ds1, ds2 float64 [R, n]."""

    def __init__(self, k1, k2, w1, ds1, ds2, n_fallback):
        self.k1, self.k2, self.w1, self.ds1, self.ds2 = k1, k2, w1, ds1, ds2
        self.n_fallback = n_fallback


def select(grid, dirs, r_exp: float = 7.0) -> Selection:
    """Two-Delaunay-line upwind selection and weights for every ray and site (Eq. 5-6)."""
    dirs = _c(dirs, np.float64)
    R = dirs.shape[0]
    n = grid.n
    xyz = _c(grid.xyz, np.float64)
    ptr = _c(grid.nbr_ptr, np.int64)
    idx = _c(grid.nbr_idx, np.int32)
    sh = _c(grid.nbr_shift, np.int8)
    wall = _c(grid.wall, np.uint8)
    L = np.asarray(grid.hi, np.float64) - np.asarray(grid.lo, np.float64)
    Lx, Ly = (float(L[0]), float(L[1])) if grid.periodic_xy else (0.0, 0.0)
    k1 = np.empty((R, n), np.int32)
    k2 = np.empty((R, n), np.int32)
    w1 = np.empty((R, n), np.float64)
    ds1 = np.empty((R, n), np.float64)
    ds2 = np.empty((R, n), np.float64)
    nfb = np.zeros(R, np.int64)
    st = lib().orc_select(n, _p(xyz, _d), _p(ptr, _i64), _p(idx, _i32), _p(sh, _i8), _p(wall, _u8), Lx, Ly, R,
                          _p(dirs, _d), float(r_exp), _p(k1, _i32), _p(k2, _i32), _p(w1, _d), _p(ds1, _d),
                          _p(ds2, _d), _p(nfb, _i64))
    if st != 0:
        raise ValueError(f"orc_select failed with status {st}")
    return Selection(k1, k2, w1, ds1, ds2, nfb)


def levels(grid, dirs, sel: Selection):
    """Per-ray level, order (sites sorted by (level, index)) and level_ptr."""
    dirs = _c(dirs, np.float64)
    R = dirs.shape[0]
    n = grid.n
    xyz = _c(grid.xyz, np.float64)
    level = np.empty((R, n), np.int32)
    order = np.empty((R, n), np.int32)
    lptr = np.zeros((R, n + 1), np.int32)
    nlev = np.empty(R, np.int32)
    st = lib().orc_levels(n, _p(xyz, _d), R, _p(dirs, _d), _p(sel.k1, _i32), _p(sel.k2, _i32), _p(level, _i32),
                          _p(order, _i32), _p(lptr, _i32), _p(nlev, _i32))
    if st != 0:
        raise ValueError(f"orc_levels failed with status {st}")
    ptrs = [lptr[r, : nlev[r] + 1].copy() for r in range(R)]
    return level, order, ptrs, nlev


# ----------------------------------------------------------------------------
# formal solutions
# ----------------------------------------------------------------------------

def fs_voronoi(grid, dirs, ray_w, sel: Selection, chi, S, I_bottom, I_top=None, keep_I: bool = False):
    """J [n, nl] (and I [R, n, nl] if keep_I) on the Voronoi grid."""
    dirs = _c(dirs, np.float64)
    ray_w = _c(ray_w, np.float64)
    chi = _c(chi, np.float64)
    S = _c(S, np.float64)
    n = grid.n
    if chi.ndim == 1:
        chi = chi[:, None]
        S = S.reshape(n, -1)
    nl = chi.shape[1]
    I_bottom = _c(np.broadcast_to(I_bottom, (n, nl)) if np.ndim(I_bottom) else np.full((n, nl), I_bottom), np.float64)
    It = None if I_top is None else _c(np.broadcast_to(I_top, (n, nl)), np.float64)
    R = dirs.shape[0]
    J = np.empty((n, nl), np.float64)
    I = np.empty((R, n, nl), np.float64) if keep_I else None
    st = lib().orc_fs_voronoi(n, R, nl, _p(_c(grid.xyz, np.float64), _d), _p(dirs, _d), _p(ray_w, _d),
                              _p(sel.k1, _i32), _p(sel.k2, _i32), _p(sel.w1, _d), _p(sel.ds1, _d),
                              _p(sel.ds2, _d), _p(chi, _d), _p(S, _d), _p(I_bottom, _d), _p(It, _d),
                              _p(I, _d), _p(J, _d))
    if st != 0:
        raise MemoryError("orc_fs_voronoi failed")
    return (J, I) if keep_I else J


def lambda_diag(grid, dirs, ray_w, sel: Selection, chi):
    """Diagonal of the Lambda operator, dJ_i/dS_i [n, nl] (orc_lambda_diag)."""
    ray_w = _c(ray_w, np.float64)
    chi = _c(chi, np.float64)
    n = grid.n
    if chi.ndim == 1:
        chi = chi[:, None]
    nl = chi.shape[1]
    out = np.empty((n, nl), np.float64)
    lib().orc_lambda_diag(n, len(ray_w), nl, _p(ray_w, _d), _p(sel.k1, _i32), _p(sel.k2, _i32), _p(sel.w1, _d),
                          _p(sel.ds1, _d), _p(sel.ds2, _d), _p(chi, _d), _p(out, _d))
    return out


def fs_regular(nx, ny, z, dx, dy, dirs, ray_w, chi, S, I_bottom, I_top=None, keep_I: bool = False):
    """J [n, nl] (and I) for short characteristics on a regular grid, fields [z][y][x][nl]."""
    z = _c(z, np.float64)
    nz = len(z)
    n = nx * ny * nz
    dirs = _c(dirs, np.float64)
    ray_w = _c(ray_w, np.float64)
    chi = _c(chi, np.float64).reshape(n, -1)
    S = _c(S, np.float64).reshape(n, -1)
    nl = chi.shape[1]
    I_bottom = _c(np.broadcast_to(I_bottom, (n, nl)) if np.ndim(I_bottom) else np.full((n, nl), I_bottom), np.float64)
    It = None if I_top is None else _c(np.broadcast_to(I_top, (n, nl)), np.float64)
    R = dirs.shape[0]
    J = np.empty((n, nl), np.float64)
    I = np.empty((R, n, nl), np.float64) if keep_I else None
    st = lib().orc_fs_regular(nx, ny, nz, float(dx), float(dy), _p(z, _d), R, _p(dirs, _d), _p(ray_w, _d), nl,
                              _p(chi, _d), _p(S, _d), _p(I_bottom, _d), _p(It, _d), _p(I, _d), _p(J, _d))
    if st != 0:
        raise MemoryError("orc_fs_regular failed")
    return (J, I) if keep_I else J


def bezier_weights(x: float):
    """(e^-x, alpha, beta, gamma) of the quadratic Bezier segment: I = e^-x I_u +
    alpha S_u + beta S_0 + gamma C."""
    E, a, b, c = (ctypes.c_double() for _ in range(4))
    lib().orc_bezier_weights(float(x), ctypes.byref(E), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return E.value, a.value, b.value, c.value


def select_downwind(grid, dirs, r_exp: float = 7.0) -> Selection:
    """Downwind lines of every ray and site: the upwind selection of the opposite directions."""
    return select(grid, -np.asarray(dirs, np.float64), r_exp)


def fs_voronoi_bezier(grid, dirs, ray_w, sel: Selection, down: Selection, chi, S, I_bottom, I_top=None,
                      keep_I: bool = False):
    """J [n, nl] (and I) on the Voronoi grid with the quadratic Bezier segment."""
    dirs = _c(dirs, np.float64)
    ray_w = _c(ray_w, np.float64)
    chi = _c(chi, np.float64)
    S = _c(S, np.float64)
    n = grid.n
    if chi.ndim == 1:
        chi = chi[:, None]
        S = S.reshape(n, -1)
    nl = chi.shape[1]
    I_bottom = _c(np.broadcast_to(I_bottom, (n, nl)) if np.ndim(I_bottom) else np.full((n, nl), I_bottom), np.float64)
    It = None if I_top is None else _c(np.broadcast_to(I_top, (n, nl)), np.float64)
    R = dirs.shape[0]
    J = np.empty((n, nl), np.float64)
    I = np.empty((R, n, nl), np.float64) if keep_I else None
    st = lib().orc_fs_voronoi_bezier(n, R, nl, _p(_c(grid.xyz, np.float64), _d), _p(dirs, _d), _p(ray_w, _d),
                                     _p(sel.k1, _i32), _p(sel.k2, _i32), _p(sel.w1, _d), _p(sel.ds1, _d),
                                     _p(sel.ds2, _d), _p(down.k1, _i32), _p(down.k2, _i32), _p(down.w1, _d),
                                     _p(down.ds1, _d), _p(down.ds2, _d), _p(chi, _d), _p(S, _d), _p(I_bottom, _d),
                                     _p(It, _d), _p(I, _d), _p(J, _d))
    if st != 0:
        raise MemoryError("orc_fs_voronoi_bezier failed")
    return (J, I) if keep_I else J


def planck(lam, T) -> float:
    """B_lambda(T) in kW m^-2 nm^-1 sr^-1 (lam in metres)."""
    return lib().orc_planck(float(lam), float(T))


def dplanck_dT(lam, T) -> float:
    return lib().orc_dplanck_dT(float(lam), float(T))


def lte(lam, kappa0, T, rho):
    """Grey LTE continuum: chi = kappa0 rho^2 T^9 and S = B_lambda(T), each [n, nl]."""
    lam = _c(np.atleast_1d(lam), np.float64)
    T = _c(T, np.float64)
    rho = _c(rho, np.float64)
    n = len(T)
    nl = len(lam)
    chi = np.empty((n, nl), np.float64)
    S = np.empty((n, nl), np.float64)
    lib().orc_lte(n, nl, _p(lam, _d), float(kappa0), _p(T, _d), _p(rho, _d), _p(chi, _d), _p(S, _d))
    return chi, S


def emergent_sites(grid, dirs):
    """Per ray, the sites whose cell touches the downwind z-wall (top for upward rays)."""
    out = []
    for d in np.asarray(dirs):
        bit = 2 if d[2] > 0 else 1
        out.append(np.nonzero(np.asarray(grid.wall) & bit)[0].astype(np.int32))
    return out


# ----------------------------------------------------------------------------
# final synthesis: back-interpolation to a regular grid and vertical rays
# ----------------------------------------------------------------------------

def regular_points(nx, ny, dx, dy, z):
    """Points (i dx, j dy, z_k) of a regular grid as [nx ny nz, 3], row (k ny + j) nx + i."""
    z = _c(z, np.float64)
    x = np.arange(nx, dtype=np.float64) * float(dx)
    y = np.arange(ny, dtype=np.float64) * float(dy)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def idw2(xyz, pts, lo, hi, periodic_xy=True, power: float = 1.0):
    """Two nearest sites of every point and the inverse-distance weight of the
    nearer one (orc_idw2, brute force). Returns idx int32 [m, 2], w1 [m] and
    the squared distances d2 [m, 2]."""
    xyz = _c(xyz, np.float64)
    pts = _c(pts, np.float64).reshape(-1, 3)
    L = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    m = pts.shape[0]
    idx = np.empty((m, 2), np.int32)
    w1 = np.empty(m, np.float64)
    d2 = np.empty((m, 2), np.float64)
    lib().orc_idw2(xyz.shape[0], _p(xyz, _d), m, _p(pts, _d), 1 if periodic_xy else 0, float(L[0]), float(L[1]),
                   float(power), _p(idx, _i32), _p(w1, _d), _p(d2, _d))
    return idx, w1, d2


def idw_apply(idx, w1, f):
    """Interpolated values w1 f[i1] + (1 - w1) f[i2] (f [n] or [n, k])."""
    f = np.asarray(f, np.float64)
    w = w1 if f.ndim == 1 else w1[:, None]
    return w * f[idx[:, 0]] + (1.0 - w) * f[idx[:, 1]]


def lc_vertical(ncol, z, chi, S, I_bottom):
    """Intensity at the top of each vertical column at mu = 1 (orc_lc_vertical):
    chi, S [nz * ncol, nl], I_bottom [ncol, nl]; returns [ncol, nl]."""
    z = _c(z, np.float64)
    nz = len(z)
    chi = _c(chi, np.float64).reshape(nz * ncol, -1)
    S = _c(S, np.float64).reshape(nz * ncol, -1)
    nl = chi.shape[1]
    Ib = _c(np.broadcast_to(I_bottom, (ncol, nl)), np.float64)
    out = np.empty((ncol, nl), np.float64)
    lib().orc_lc_vertical(ncol, nz, nl, _p(z, _d), _p(chi, _d), _p(S, _d), _p(Ib, _d), _p(out, _d))
    return out


# ----------------------------------------------------------------------------
# reverse-mode derivatives
# ----------------------------------------------------------------------------

def fs_voronoi_vjp(grid, dirs, ray_w, sel: Selection, chi, S, I, dL_dI=None, dL_dJ=None):
    """(dL/dchi, dL/dS, dL/dI_bottom, dL/dI_top), each [n, nl], for the forward
    intensities I [R, n, nl] of ``fs_voronoi(..., keep_I=True)``."""
    dirs = _c(dirs, np.float64)
    ray_w = _c(ray_w, np.float64)
    chi = _c(chi, np.float64)
    S = _c(S, np.float64)
    I = _c(I, np.float64)
    R, n, nl = I.shape
    gI = None if dL_dI is None else _c(dL_dI, np.float64)
    gJ = None if dL_dJ is None else _c(dL_dJ, np.float64)
    out = [np.empty((n, nl), np.float64) for _ in range(4)]
    st = lib().orc_fs_voronoi_vjp(n, R, nl, _p(_c(grid.xyz, np.float64), _d), _p(dirs, _d), _p(ray_w, _d),
                                  _p(sel.k1, _i32), _p(sel.k2, _i32), _p(sel.w1, _d), _p(sel.ds1, _d),
                                  _p(sel.ds2, _d), _p(chi, _d), _p(S, _d), _p(I, _d), _p(gI, _d), _p(gJ, _d),
                                  *[_p(o, _d) for o in out])
    if st != 0:
        raise MemoryError("orc_fs_voronoi_vjp failed")
    return tuple(out)


def lte_vjp(lam, kappa0, T, rho, g_chi, g_S, g_Ib=None):
    """(dL/dT, dL/drho) [n] through chi = kappa0 rho^2 T^9 and S = I_bottom = B_lambda(T)."""
    lam = _c(np.atleast_1d(lam), np.float64)
    T = _c(T, np.float64)
    rho = _c(rho, np.float64)
    n = len(T)
    gT = np.empty(n, np.float64)
    gr = np.empty(n, np.float64)
    lib().orc_lte_vjp(n, len(lam), _p(lam, _d), float(kappa0), _p(T, _d), _p(rho, _d),
                      _p(_c(g_chi, np.float64), _d), _p(_c(g_S, np.float64), _d),
                      None if g_Ib is None else _p(_c(g_Ib, np.float64), _d), _p(gT, _d), _p(gr, _d))
    return gT, gr


def emergent_loss(grid, dirs, ray_w, sel, lam, kappa0, T, rho, target=None):
    """L = sum over upward rays and their top-wall sites of (I - target)^2 for the
    grey LTE continuum, with its gradient (dL/dT, dL/drho) by the reverse sweep.
    target: dict ray -> [sites, nl] array (None: zero)."""
    chi, S = lte(lam, kappa0, T, rho)
    J, I = fs_voronoi(grid, dirs, ray_w, sel, chi, S, S, keep_I=True)
    em = emergent_sites(grid, dirs)
    gI = np.zeros_like(I)
    L = 0.0
    for r in range(len(dirs)):
        if dirs[r, 2] <= 0:
            continue
        tr = 0.0 if target is None else target[r]
        d = I[r, em[r]] - tr
        L += float(np.sum(d * d))
        gI[r, em[r]] = 2.0 * d
    g_chi, g_S, g_Ib, _ = fs_voronoi_vjp(grid, dirs, ray_w, sel, chi, S, I, dL_dI=gI)
    gT, gr = lte_vjp(lam, kappa0, T, rho, g_chi, g_S, g_Ib)
    return L, gT, gr, I
