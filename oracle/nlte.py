"""Two-level-atom Lambda iteration on the oracle side (FP64, numpy + the C sweep).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sect. 2.1: the line source function of a two-level atom under complete
redistribution is S_L = (1 - eps) Jbar + eps B (Eq. 3 with the profile-weighted
mean intensity Jbar), J = Lambda[S] is one formal solution over all rays (Eq.
4), and the plain Lambda iteration alternates the two until the largest
relative change of S_L drops below a tolerance (about 1e-3, Sect. 3.3). The
accelerated variant divides each correction by 1 - (1 - eps) Lbar*, with Lbar*
the diagonal of the line operator (the local, Jacobi operator).

With a grey continuum of opacity chi_c and thermal source B beside the line of
opacity chi_L phi_lambda, the total opacity and source at each wavelength are
chi = chi_c + chi_L phi and S = (chi_L phi S_L + chi_c B) / chi. The profile
weights satisfy sum_lambda wlam * phi = 1 at every site (the caller normalises
them), so S_L = B is an exact fixed point of an isothermal, thermalised box.
"""

from __future__ import annotations

import numpy as np

from . import fs_voronoi, fs_voronoi_bezier, idw2, idw_apply, lambda_diag, lc_vertical, regular_points


def assemble(chi_c, chi_L, phi, B, S_L):
    """Total opacity and source [n, nl] from the continuum and the line (Sect. 2.1, Eq. 3)."""
    chi = chi_c[:, None] + chi_L[:, None] * phi
    S = (chi_L[:, None] * phi * S_L[:, None] + chi_c[:, None] * B[:, None]) / chi
    return chi, S


def jbar(phi, wlam, J):
    """Profile-weighted mean intensity sum_lambda wlam phi J."""
    return np.sum(wlam[None, :] * phi * J, axis=1)


def lambda_step(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, S_L, I_top=None, down=None):
    """One Lambda iteration: returns (S_L new, max relative change). With the
    downwind lines ``down`` the formal solution uses the quadratic Bezier
    segment instead of the linear one."""
    chi, S = assemble(chi_c, chi_L, phi, B, S_L)
    nl = phi.shape[1]
    Ib = np.repeat(B[:, None], nl, axis=1)
    It = None if I_top is None else np.repeat(np.asarray(I_top)[:, None], nl, axis=1)
    if down is None:
        J = fs_voronoi(grid, dirs, ray_w, sel, chi, S, Ib, I_top=It)
    else:
        J = fs_voronoi_bezier(grid, dirs, ray_w, sel, down, chi, S, Ib, I_top=It)
    S_new = (1.0 - eps) * jbar(phi, wlam, J) + eps * B
    dS = float(np.max(np.abs(S_new - S_L) / np.abs(S_L)))
    return S_new, dS


def line_diag(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam):
    """Diagonal of the line operator, dJbar_i/dS_L,i = sum_lambda wlam phi (chi_L phi / chi) Lambda*_ii:
    S_L,i enters S_lambda,i with the weight chi_L phi / chi (Eq. 3 with the
    continuum), and Lambda*_ii carries it to J_lambda,i."""
    chi = chi_c[:, None] + chi_L[:, None] * phi
    Ld = lambda_diag(grid, dirs, ray_w, sel, chi)
    return np.sum(wlam[None, :] * phi * (chi_L[:, None] * phi / chi) * Ld, axis=1)


def ali_step(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, S_L, Lbar, I_top=None):
    """One Jacobi-accelerated step: S_L + [(1 - eps) Jbar + eps B - S_L] / [1 - (1 - eps) Lbar]."""
    chi, S = assemble(chi_c, chi_L, phi, B, S_L)
    nl = phi.shape[1]
    Ib = np.repeat(B[:, None], nl, axis=1)
    It = None if I_top is None else np.repeat(np.asarray(I_top)[:, None], nl, axis=1)
    J = fs_voronoi(grid, dirs, ray_w, sel, chi, S, Ib, I_top=It)
    S_fs = (1.0 - eps) * jbar(phi, wlam, J) + eps * B
    S_new = S_L + (S_fs - S_L) / (1.0 - (1.0 - eps) * Lbar)
    dS = float(np.max(np.abs(S_new - S_L) / np.abs(S_L)))
    return S_new, dS


def lambda_iterate(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, max_iter=1000, tol=1e-3,
                   S_start=None, I_top=None, accel=False, down=None):
    """Lambda iteration from S_L = B (or ``S_start``) until max dS/S < tol:
    plain, or with the Jacobi (local-operator) acceleration when ``accel``;
    the plain one with the quadratic Bezier segment when ``down`` (the
    downwind lines) is given.

    Returns (S_L, history of dS, number of iterations done, converged flag).
    """
    if accel and down is not None:
        raise ValueError("the accelerated iteration uses the linear segment")
    S_L = np.array(B if S_start is None else S_start, dtype=np.float64)
    Lbar = line_diag(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam) if accel else None
    hist = []
    for it in range(max_iter):
        if accel:
            S_L, dS = ali_step(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, S_L, Lbar, I_top)
        else:
            S_L, dS = lambda_step(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, S_L, I_top, down)
        hist.append(dS)
        if not np.isfinite(dS):
            raise FloatingPointError("non-finite source-function change")
        if dS < tol:
            return S_L, np.array(hist), it + 1, True
    return S_L, np.array(hist), max_iter, False


def jbar_matrix(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, I_top=None, groups=None):
    """The affine map of the line source function to Jbar for fixed opacities,
    Jbar = M S_L + c: c is Jbar at S_L = 0 and column j of M is Jbar(e_j) - c
    (one formal solution per column). ``groups`` (optional list of index
    arrays) ties sites that share one unknown, e.g. the sites of one plane of a
    horizontally uniform column. Returns (M, c at the group representatives,
    the representatives)."""
    n = grid.n
    nl = phi.shape[1]
    Ib = np.repeat(B[:, None], nl, axis=1)
    It = None if I_top is None else np.repeat(np.asarray(I_top)[:, None], nl, axis=1)

    def jb(S_L):
        chi, S = assemble(chi_c, chi_L, phi, B, S_L)
        return jbar(phi, wlam, fs_voronoi(grid, dirs, ray_w, sel, chi, S, Ib, I_top=It))

    if groups is None:
        groups = [np.array([i]) for i in range(n)]
    m = len(groups)
    c = jb(np.zeros(n))
    M = np.empty((m, m))
    rep = np.array([g[0] for g in groups])
    for j, gidx in enumerate(groups):
        e = np.zeros(n)
        e[gidx] = 1.0
        M[:, j] = (jb(e) - c)[rep]
    return M, c[rep], rep


def dense_fixed_point(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, eps, I_top=None, groups=None):
    """Fixed point of the Lambda iteration by a dense linear solve of
    (1 - (1 - eps) M) S = (1 - eps) c + eps B (see jbar_matrix)."""
    n = grid.n
    if groups is None:
        groups = [np.array([i]) for i in range(n)]
    M, c, rep = jbar_matrix(grid, dirs, ray_w, sel, chi_c, chi_L, phi, wlam, B, I_top=I_top, groups=groups)
    m = len(groups)
    A = np.eye(m) - (1.0 - eps) * M
    rhs = (1.0 - eps) * c + eps * B[rep]
    sol = np.linalg.solve(A, rhs)
    S = np.empty(n)
    for j, gidx in enumerate(groups):
        S[gidx] = sol[j]
    return S


def synthesize(grid, S_line, nx, ny, dx, dy, z, phi, chi_L, chi_c, B, power=1.0, I_bottom=None):
    """Emergent line intensity at mu = 1 on a regular grid from a solution on a
    Voronoi grid (Sect. 2.5, closing paragraph): S_line on the sites is carried
    to the regular points by inverse-distance weights of the two nearest sites,
    the line and continuum are assembled there (phi [m, nl], chi_L, chi_c, B
    [m], m = nx ny nz in row order (k ny + j) nx + i), and each column is
    integrated upwards from I_bottom (default B of the bottom plane). Returns
    the top-plane intensities [nx ny, nl]."""
    z = np.asarray(z, np.float64)
    pts = regular_points(nx, ny, dx, dy, z)
    idx, w1, _ = idw2(grid.xyz, pts, grid.lo, grid.hi, grid.periodic_xy, power)
    S_reg = idw_apply(idx, w1, S_line)
    chi, S = assemble(chi_c, chi_L, phi, B, S_reg)
    ncol = nx * ny
    if I_bottom is None:
        I_bottom = np.repeat(B[:ncol, None], phi.shape[1], axis=1)
    return lc_vertical(ncol, z, chi, S, I_bottom)
