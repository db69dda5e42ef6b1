"""Pins of the oracle's final-synthesis routines (Sect. 2.5, closing paragraph;
Sect. 3.2): two-nearest-site inverse-distance interpolation from a Voronoi grid
to a regular grid, and long characteristics along vertical columns at mu = 1.

The nearest-site search is checked against scipy's k-d tree (an independent
library routine, periodic through its box size); the weights against closed
forms (power 1 on a segment is linear interpolation); the column integration
against the exact emergent intensity of a source linear in optical depth, the
isothermal box and the regular-grid short-characteristics oracle on its one
vertical ray (no interpolation happens at mu = 1, so the two must agree).
"""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from oracle import nlte as onl
from synth.nlte import line_setup


def _box(rng, n_sites, n_pts):
    lo = np.array([0.0, 0.0, -0.5])
    L = np.array([6.0, 6.0, 3.0])
    return lo, lo + L, lo + rng.random((n_sites, 3)) * L, lo + rng.random((n_pts, 3)) * L


@pytest.mark.parametrize("periodic", [True, False])
def test_idw2_nearest_sites_match_kdtree(periodic):
    rng = np.random.default_rng(5)
    lo, hi, xyz, pts = _box(rng, 3000, 2000)
    # points close to the periodic walls, where the minimum image matters
    pts[:200, 0] = lo[0] + 1e-3 * rng.random(200)
    pts[200:400, 1] = hi[1] - 1e-3 * rng.random(200)
    idx, w1, d2 = oracle.idw2(xyz, pts, lo, hi, periodic)
    L = hi - lo
    if periodic:
        tree = cKDTree(xyz - lo, boxsize=[L[0], L[1], 10 * L[2]])  # z never wraps
        dist, ii = tree.query(pts - lo, k=2)
    else:
        dist, ii = cKDTree(xyz).query(pts, k=2)
    assert np.array_equal(idx, ii.astype(np.int32))
    np.testing.assert_allclose(np.sqrt(d2), dist, rtol=1e-13, atol=0)
    assert np.all(d2[:, 0] <= d2[:, 1])
    assert np.all((w1 >= 0.5) & (w1 <= 1.0))  # the nearer site weighs at least as much


@pytest.mark.parametrize("power", [1.0, 2.0, 3.5])
def test_idw_weights_closed_form_on_a_segment(power):
    """Two sites on a vertical line, points between them: u_k = d_k^-p; for
    p = 1 the interpolant is the straight line through the two values."""
    a, b = -0.25, 1.75
    xyz = np.array([[1.0, 2.0, a], [1.0, 2.0, b]])
    zq = np.linspace(a, b, 41)
    pts = np.stack([np.full_like(zq, 1.0), np.full_like(zq, 2.0), zq], 1)
    f = np.array([3.0, -5.0])
    idx, w1, d2 = oracle.idw2(xyz, pts, [0, 0, -1], [6, 6, 2], False, power)
    val = oracle.idw_apply(idx, w1, f)
    da, db = zq - a, b - zq
    with np.errstate(divide="ignore", invalid="ignore"):
        exact = np.where(da == 0, f[0], np.where(db == 0, f[1],
                         (f[0] * da ** -power + f[1] * db ** -power) / (da ** -power + db ** -power)))
    np.testing.assert_allclose(val, exact, rtol=1e-14, atol=1e-14)
    if power == 1.0:
        np.testing.assert_allclose(val, f[0] + (f[1] - f[0]) * da / (b - a), rtol=1e-14, atol=1e-14)


def test_idw_exact_at_sites_single_site_and_ties():
    rng = np.random.default_rng(7)
    lo, hi, xyz, _ = _box(rng, 500, 0)
    pick = rng.choice(500, 50, replace=False)
    idx, w1, d2 = oracle.idw2(xyz, xyz[pick], lo, hi, True, 1.0)
    assert np.array_equal(idx[:, 0], pick.astype(np.int32))
    assert np.all(w1 == 1.0) and np.all(d2[:, 0] == 0.0) and np.all(d2[:, 1] > 0.0)
    f = rng.random(500)
    assert np.array_equal(oracle.idw_apply(idx, w1, f), f[pick])
    # one site: both neighbours are that site, weight 1
    idx, w1, _ = oracle.idw2(xyz[:1], xyz[1:10], lo, hi, True)
    assert np.all(idx == 0) and np.all(w1 == 1.0)
    # equidistant sites: the smaller index is the first neighbour, equal weights
    two = np.array([[3.0, 3.0, 0.0], [3.0, 3.0, 1.0], [1.0, 1.0, 0.5]])
    idx, w1, _ = oracle.idw2(two[[1, 0, 2]], np.array([[3.0, 3.0, 0.5]]), lo, hi, True)
    assert idx.tolist() == [[0, 1]] and w1[0] == 0.5


def test_idw_apply_preserves_constants_and_bounds():
    rng = np.random.default_rng(8)
    lo, hi, xyz, pts = _box(rng, 800, 3000)
    idx, w1, _ = oracle.idw2(xyz, pts, lo, hi, True, 1.0)
    np.testing.assert_allclose(oracle.idw_apply(idx, w1, np.full(800, 2.5)), 2.5, rtol=1e-15)
    f = rng.standard_normal((800, 3))
    v = oracle.idw_apply(idx, w1, f)
    lo_v = np.minimum(f[idx[:, 0]], f[idx[:, 1]])
    hi_v = np.maximum(f[idx[:, 0]], f[idx[:, 1]])
    assert np.all(v >= lo_v - 1e-15) and np.all(v <= hi_v + 1e-15)


def _columns(rng, ncol, nz):
    z = np.cumsum(rng.uniform(0.5, 1.5, nz))
    chi = np.exp(rng.uniform(-3.0, 1.0, (nz * ncol, 1)))
    return z, chi


def test_lc_vertical_exact_for_source_linear_in_tau():
    """S = a + b tau (tau from the top, trapezoid optical depth) with the
    diffusion boundary I_bottom = a + b (tau_bottom + 1) emerges as a + b."""
    rng = np.random.default_rng(9)
    ncol, nz = 12, 60
    z, chi = _columns(rng, ncol, nz)
    chi = np.repeat(chi, 3, axis=1) * np.array([0.3, 1.0, 4.0])  # three wavelengths
    c3 = chi.reshape(nz, ncol, 3)
    dtau = 0.5 * (c3[1:] + c3[:-1]) * np.diff(z)[:, None, None]
    tau = np.concatenate([np.cumsum(dtau[::-1], axis=0)[::-1], np.zeros((1, ncol, 3))], axis=0)
    a, b = 0.7, 1.3
    S = a + b * tau
    Ib = a + b * (tau[0] + 1.0)
    out = oracle.lc_vertical(ncol, z, chi, S.reshape(nz * ncol, 3), Ib)
    np.testing.assert_allclose(out, a + b, rtol=1e-12)


def test_lc_vertical_isothermal_and_matches_regular_oracle():
    rng = np.random.default_rng(10)
    nx, ny, nz, nl = 5, 4, 30, 2
    ncol = nx * ny
    z, chi = _columns(rng, ncol, nz)
    chi = np.repeat(chi, nl, axis=1)
    out = oracle.lc_vertical(ncol, z, chi, np.full((nz * ncol, nl), 2.0), np.full((ncol, nl), 2.0))
    np.testing.assert_allclose(out, 2.0, rtol=1e-14)
    S = rng.uniform(0.5, 2.0, (nz * ncol, nl))
    Ib = rng.uniform(0.5, 2.0, (ncol, nl))
    out = oracle.lc_vertical(ncol, z, chi, S, Ib)
    Ib_full = np.zeros((nz * ncol, nl))
    Ib_full[:ncol] = Ib
    _, I = oracle.fs_regular(nx, ny, z, 1.0, 1.0, np.array([[0.0, 0.0, 1.0]]), np.array([1.0]), chi, S, Ib_full,
                             keep_I=True)
    np.testing.assert_allclose(out, I[0, (nz - 1) * ncol:], rtol=1e-13)


def test_synthesis_identity_on_lattice_and_isothermal():
    """Sites on the regular points: the interpolation is the identity, so the
    synthesis equals the column integration of the assembled line at the sites;
    an isothermal box with S_line = B emerges as B."""
    rng = np.random.default_rng(11)
    nx, ny, nz = 4, 3, 12
    dx, dy = 0.5, 0.5
    z = np.cumsum(rng.uniform(0.05, 0.15, nz)) - 0.5
    g = synth.lattice_grid(nx, ny, z, dx, dy)
    m = nx * ny * nz
    T = 5000.0 + 500.0 * rng.random(m)
    rho = 1e-4 * np.exp(-np.repeat(z, nx * ny) / 0.3)
    line = line_setup(T, rho, n_lambda=9)
    chi_L = line.chi_line * 1e6
    chi_c = np.full(m, 3.0)
    B = rng.uniform(1.0, 2.0, m)
    S_line = rng.uniform(0.5, 1.5, m)
    out = onl.synthesize(g, S_line, nx, ny, dx, dy, z, line.phi, chi_L, chi_c, B)
    chi, S = onl.assemble(chi_c, chi_L, line.phi, B, S_line)
    ref = oracle.lc_vertical(nx * ny, z, chi, S, np.repeat(B[: nx * ny, None], 9, axis=1))
    assert np.array_equal(out, ref)
    Bc = np.full(m, 1.7)
    out = onl.synthesize(g, Bc, nx, ny, dx, dy, z, line.phi, chi_L, chi_c, Bc)
    np.testing.assert_allclose(out, 1.7, rtol=1e-14)
