"""Formal solution on Voronoi and regular grids (Sect. 2.1 Eq. 1-2, 4; Sect. 2.5 Eq. 5; Sect. 2.6).

Pins (closed forms and limits that any correct discretisation with S linear
along segments must reproduce):
* isothermal medium: S = I_bottom = B everywhere gives I = B on every upward
  ray, for any opacity (weights sum to one and e^-x + Psi_u + Psi_0 = 1);
* source linear in optical depth along vertical lines:
  I_em = a + b (1 - e^-tau_max) at mu = 1 when I_bottom = S(tau_max);
* regular grid, horizontally uniform, any mu: I_em = a + b mu (1 - e^-tau_max/mu);
* optically thin: chi = 0 carries I_bottom unchanged; chi -> s chi gives
  (I - I_bc)/s -> the trapezoid emission integral along the chosen lines;
* a Voronoi grid built on a lattice equals the regular grid solver for
  vertical rays, for arbitrary fields;
* exact integer shifts on a regular grid transport a pattern unchanged;
* the angle quadrature of an isotropic field returns the field.
"""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def recipe():
    atm = synth.make_atmosphere(2000, seed=21)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    return atm, g, dirs, w


def _rel(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


def test_isothermal_gives_I_equals_B(orc, recipe):
    atm, g, dirs, w = recipe
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(0)
    nl = 3
    chi = 10.0 ** rng.uniform(-8, -3, size=(g.n, nl))
    B = np.array([2.5, 7.0, 31.0])
    S = np.broadcast_to(B, (g.n, nl)).copy()
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, S, keep_I=True)
    up = dirs[:, 2] > 0
    assert _rel(I[up], S[None]) < 1e-14
    # with I_top = B as well, every ray and J equal B
    J2, I2 = orc.fs_voronoi(g, dirs, w, sel, chi, S, S, I_top=S, keep_I=True)
    assert _rel(I2, S[None]) < 1e-14
    assert _rel(J2, S) < 1e-14
    # with I_top = 0: downward I reaches B where the optical depth from the top exceeds 40
    # (every path from the top wall to a site 1 Mm down crosses at least 1 Mm * chi = 400)
    chi_thick = np.full((g.n, nl), 4e-4)
    J3, I3 = orc.fs_voronoi(g, dirs, w, sel, chi_thick, S, S, keep_I=True)
    deep = g.xyz[:, 2] < atm.box.hi[2] - 1.0e6
    assert deep.sum() > 100
    assert _rel(I3[~up][:, deep], S[None, deep]) < 1e-12


def test_linear_source_on_vertical_chains(orc):
    # lattice with uneven z spacing; every upward ray is carried along vertical lines
    z = np.cumsum(np.r_[0.0, np.random.default_rng(1).uniform(0.2, 2.0, 40)])
    g = synth.lattice_grid(3, 2, z)
    dirs, w = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    chi0 = 0.37
    ztop = z[-1]
    tau = chi0 * (ztop - g.xyz[:, 2])
    tau_max = chi0 * (ztop - z[0])
    a, b = 1.7, 0.45
    S = (a + b * tau)[:, None]
    chi = np.full_like(S, chi0)
    Ib = np.full_like(S, a + b * tau_max)
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, keep_I=True)
    top = g.xyz[:, 2] == ztop
    want = a + b * (1.0 - np.exp(-tau_max))
    for r in np.nonzero(dirs[:, 2] > 0)[0]:
        assert np.max(np.abs(I[r, top, 0] - want)) / want < 1e-12
    # and at every height the exact solution of that depth:
    # I(t) = (a + b tau_max) e^-(tau_max - t) + int_t^tau_max (a + b s) e^-(s - t) ds
    dt = tau_max - tau
    exact = (a + b * tau_max) * np.exp(-dt) + a * (1 - np.exp(-dt)) + b * (tau + 1 - (tau_max + 1) * np.exp(-dt))
    r0 = int(np.nonzero(dirs[:, 2] > 0)[0][0])
    assert np.max(np.abs(I[r0, :, 0] - exact) / exact) < 1e-12


def test_regular_linear_source_any_mu(orc):
    nx, ny = 5, 4
    z = np.cumsum(np.r_[0.0, np.random.default_rng(2).uniform(0.05, 0.3, 60)])
    dirs, w = synth.gauss_legendre_quadrature()
    chi0 = 1.3
    ztop = z[-1]
    zz = np.repeat(z, nx * ny)
    tau = chi0 * (ztop - zz)
    tau_max = chi0 * (ztop - z[0])
    a, b = 0.8, 2.2
    S = (a + b * tau)[:, None]
    chi = np.full_like(S, chi0)
    Ib = np.full_like(S, a + b * tau_max)
    J, I = orc.fs_regular(nx, ny, z, 0.3, 0.45, dirs, w, chi, S, Ib, keep_I=True)
    top = zz == ztop
    for r in np.nonzero(dirs[:, 2] > 0)[0]:
        mu = dirs[r, 2]
        want = a + b * mu * (1.0 - np.exp(-tau_max / mu))
        assert np.max(np.abs(I[r, top, 0] - want)) / want < 1e-12


def test_optically_thin_transport(orc, recipe):
    atm, g, dirs, w = recipe
    sel = orc.select(g, dirs)
    nl = 2
    chi = np.zeros((g.n, nl))
    S = np.random.default_rng(3).uniform(0, 5, (g.n, nl))
    Ib = np.full((g.n, nl), 3.25)
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, I_top=Ib, keep_I=True)
    assert np.all(np.isfinite(I))
    assert np.max(np.abs(I - 3.25)) < 4e-15 * 3.25 * 100


def _emission_integral(g, dirs, sel, chi, S):
    """D_i = sum_j w_j [D_kj + xhat_j (S_kj + S_i)/2], xhat = (chi_kj + chi_i)/2 * ds_j,
    D = 0 at boundary sites: the first-order term of I in the opacity scale."""
    R = len(dirs)
    D = np.zeros((R, g.n))
    for r in range(R):
        order = np.argsort((1 if dirs[r, 2] > 0 else -1) * g.xyz[:, 2], kind="stable")
        for i in order:
            k1, k2 = sel.k1[r, i], sel.k2[r, i]
            if k1 < 0:
                continue
            x1 = 0.5 * (chi[k1] + chi[i]) * sel.ds1[r, i]
            v = D[r, k1] + x1 * 0.5 * (S[k1] + S[i])
            if k2 >= 0:
                x2 = 0.5 * (chi[k2] + chi[i]) * sel.ds2[r, i]
                v2 = D[r, k2] + x2 * 0.5 * (S[k2] + S[i])
                v = sel.w1[r, i] * v + (1 - sel.w1[r, i]) * v2
            D[r, i] = v
    return D


def test_optically_thin_limit_is_trapezoid_emission(orc, recipe):
    atm, g, dirs, w = recipe
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(5)
    chi = rng.uniform(0.5, 2.0, g.n) / (atm.box.L[2] * 10)
    S = rng.uniform(1.0, 4.0, g.n)
    D = _emission_integral(g, dirs, sel, chi, S)
    errs = []
    for s in (1e-3, 1e-4):
        _, I = orc.fs_voronoi(g, dirs, w, sel, (s * chi)[:, None], S[:, None], 0.0, keep_I=True)
        errs.append(np.max(np.abs(I[..., 0] / s - D)) / np.max(np.abs(D)))
    assert errs[1] < errs[0] / 5 and errs[1] < 1e-3


def test_lattice_voronoi_equals_regular_for_vertical_rays(orc):
    nx, ny = 6, 5
    z = np.cumsum(np.r_[0.0, np.random.default_rng(7).uniform(0.1, 1.0, 30)])
    g = synth.lattice_grid(nx, ny, z, dx=0.7, dy=0.9)
    dirs, w = synth.vertical_quadrature()
    rng = np.random.default_rng(8)
    nl = 4
    chi = 10 ** rng.uniform(-2, 1, (g.n, nl))
    S = rng.uniform(0.1, 9.0, (g.n, nl))
    Ib = rng.uniform(0.1, 9.0, (g.n, nl))
    It = rng.uniform(0.0, 1.0, (g.n, nl))
    sel = orc.select(g, dirs)
    Jv, Iv = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, I_top=It, keep_I=True)
    Jr, Ir = orc.fs_regular(nx, ny, z, 0.7, 0.9, dirs, w, chi, S, Ib, I_top=It, keep_I=True)
    # (i*dx)/dx is not always exactly i in binary, so the regular solver's bilinear
    # weights can be 1 - 4e-16 instead of 1: agreement is to rounding, not bitwise
    assert np.max(np.abs(Iv - Ir) / np.abs(Ir)) < 1e-13
    assert np.max(np.abs(Jv - Jr) / np.abs(Jr)) < 1e-13


def test_regular_integer_shift_transport(orc):
    # dx = dy = dz and a ray with tan(theta) cos(phi) = tan(theta) sin(phi) = 1:
    # each plane is the previous one shifted by one cell in x and y
    nx, ny, nz = 7, 5, 9
    z = np.arange(nz, dtype=float)
    mu = 1.0 / np.sqrt(3.0)
    d = np.array([[mu, mu, mu]])
    w = np.array([1.0])
    rng = np.random.default_rng(9)
    pattern = rng.uniform(0, 1, (ny, nx))
    Ib = np.zeros((nz, ny, nx))
    Ib[0] = pattern
    chi = np.zeros((nz * ny * nx, 1))
    J, I = orc.fs_regular(nx, ny, z, 1.0, 1.0, d, w, chi, np.zeros_like(chi), Ib.reshape(-1, 1), keep_I=True)
    top = I[0, :, 0].reshape(nz, ny, nx)[-1]
    want = np.roll(np.roll(pattern, nz - 1, axis=0), nz - 1, axis=1)
    assert np.max(np.abs(top - want)) < 1e-12


@pytest.mark.parametrize("up", [True, False])
def test_regular_fractional_shift_fourier_mode(orc, up):
    """Bilinear interpolation at a fractional upwind offset (Sect. 2.6, linear
    interpolation in the upwind plane), pinned by its closed form. With constant
    chi, S = 0 and a boundary plane cos(k x) that is constant in y, the upwind
    point of every point lies a = p + t cells upwind in x, and linear
    interpolation of the Fourier mode e^{ikx} there gives the mode times
    e^{-ikp dx} ((1 - t) + t e^{-ik dx}); each plane also attenuates by
    e^{-chi ds}. After s planes the intensity is Re[(e^{-chi ds} G)^s e^{ikx}].
    Nearest-cell rounding or swapped weights change |G| and fail."""
    nx, ny, nz = 24, 3, 8
    dx, dy = 1.0, 0.8
    z = np.arange(nz, dtype=float)  # dz = 1
    a_x, a_y = 2.37, 0.61  # upwind offset per plane, in cells of x and of y
    mz = 1.0 / np.sqrt(1.0 + (a_x * dx) ** 2 + (a_y * dy) ** 2)
    d = np.array([[a_x * dx * mz, a_y * dy * mz, mz if up else -mz]])
    w = np.array([1.0])
    m = 3
    k = 2 * np.pi * m / (nx * dx)
    x = np.arange(nx) * dx
    plane = np.broadcast_to(np.cos(k * x)[None, :], (ny, nx))
    n = nx * ny * nz
    chi_v = 0.05
    chi = np.full((n, 1), chi_v)
    bnd = np.zeros((nz, ny, nx))
    bnd[0 if up else nz - 1] = plane
    kw = dict(keep_I=True)
    if up:
        J, I = orc.fs_regular(nx, ny, z, dx, dy, d, w, chi, np.zeros_like(chi), bnd.reshape(-1, 1), **kw)
    else:
        J, I = orc.fs_regular(nx, ny, z, dx, dy, d, w, chi, np.zeros_like(chi), np.zeros((n, 1)),
                              I_top=bnd.reshape(-1, 1), **kw)
    got = I[0, :, 0].reshape(nz, ny, nx)
    ds = 1.0 / mz
    p, t = 2, 0.37
    G = np.exp(-chi_v * ds) * np.exp(-1j * k * p * dx) * ((1 - t) + t * np.exp(-1j * k * dx))
    for s in range(nz):
        kk = s if up else nz - 1 - s
        want = np.real(G ** s * np.exp(1j * k * x))
        assert np.max(np.abs(got[kk] - want[None, :])) < 1e-13, s
    # the interpolation damps the mode: |G| < e^{-chi ds} (nearest-cell rounding would not)
    assert abs(G) < np.exp(-chi_v * ds) * 0.95


def test_regular_fractional_shift_matches_map_coordinates(orc):
    """Multi-plane optically thin transport (chi = S = 0: each plane is the
    upwind plane interpolated) of a random periodic pattern, at fractional
    offsets in both x and y with dx != dy, against scipy's periodic linear
    interpolation (map_coordinates, order 1, grid-wrap) applied plane by plane."""
    from scipy.ndimage import map_coordinates

    nx, ny, nz = 13, 11, 6
    dx, dy = 0.7, 1.3
    z = np.cumsum(np.r_[0.0, np.random.default_rng(31).uniform(0.5, 1.5, nz - 1)])  # uneven planes
    d = np.array([[0.55, -0.31, 0.0]])
    d[0, 2] = np.sqrt(1 - d[0, 0] ** 2 - d[0, 1] ** 2)
    w = np.array([1.0])
    pattern = np.random.default_rng(32).uniform(0.0, 1.0, (ny, nx))
    n = nx * ny * nz
    chi = np.zeros((n, 1))
    Ib = np.zeros((nz, ny, nx))
    Ib[0] = pattern
    J, I = orc.fs_regular(nx, ny, z, dx, dy, d, w, chi, np.zeros_like(chi), Ib.reshape(-1, 1), keep_I=True)
    got = I[0, :, 0].reshape(nz, ny, nx)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    want = pattern
    for s in range(1, nz):
        ds = (z[s] - z[s - 1]) / d[0, 2]
        coords = [jj - ds * d[0, 1] / dy, ii - ds * d[0, 0] / dx]
        want = map_coordinates(want, coords, order=1, mode="grid-wrap")
        assert np.max(np.abs(got[s] - want)) < 1e-13, s


def test_regular_isothermal(orc):
    nx, ny = 4, 4
    z = np.linspace(0, 3, 12)
    dirs, w = synth.gauss_legendre_quadrature()
    n = nx * ny * len(z)
    chi = np.random.default_rng(10).uniform(0.1, 3.0, (n, 2))
    S = np.broadcast_to([4.0, 0.5], (n, 2)).copy()
    J, I = orc.fs_regular(nx, ny, z, 0.5, 0.5, dirs, w, chi, S, S, I_top=S, keep_I=True)
    assert _rel(I, S[None]) < 1e-14 and _rel(J, S) < 1e-14


def test_lte_planck(orc):
    # Planck function against its definition in mpmath, in kW m^-2 nm^-1 sr^-1
    import mpmath as mp

    h, c, k = mp.mpf("6.62607015e-34"), mp.mpf(299792458), mp.mpf("1.380649e-23")
    for lam, T in [(500e-9, 6000.0), (400e-9, 3700.0), (900e-9, 7400.0), (121.568e-9, 4200.0)]:
        lm = mp.mpf(lam)
        B = 2 * h * c**2 / lm**5 / (mp.exp(h * c / (lm * k * T)) - 1) * mp.mpf("1e-12")
        assert abs(orc.planck(lam, T) - float(B)) / float(B) < 1e-14
        dB = mp.diff(lambda t: 2 * h * c**2 / lm**5 / (mp.exp(h * c / (lm * k * t)) - 1) * mp.mpf("1e-12"), mp.mpf(T))
        assert abs(orc.dplanck_dT(lam, T) - float(dB)) / float(dB) < 1e-13
    # solar-like continuum at 500 nm, 6000 K: about 32 kW m^-2 nm^-1 sr^-1
    assert 30 < orc.planck(500e-9, 6000.0) < 34
    chi, S = orc.lte([500e-9, 600e-9], 2.0e-33, np.array([5000.0, 6000.0]), np.array([1e-4, 2e-4]))
    assert np.allclose(chi[:, 0], chi[:, 1])
    assert abs(chi[1, 0] - 2.0e-33 * 4e-8 * 6000.0**9) / chi[1, 0] < 1e-15
