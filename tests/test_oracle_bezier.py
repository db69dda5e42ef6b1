"""Pins of the oracle's quadratic Bezier segment, the higher-order formal
solver the paper names as the way to improve its linear one (Sect. 2.5; de la
Cruz Rodriguez & Piskunov 2013).

* the weights alpha, beta, gamma against 50-digit closed forms and against the
  integrals of the Bernstein basis times e^-(x - t), and the identities
  alpha + beta + gamma = 1 - e^-x, alpha + gamma/2 = Psi_u, beta + gamma/2 = Psi_0
  (a control value at the midpoint is the linear segment);
* third-order convergence of the emergent intensity on vertical chains for
  smooth sources (monotone and oscillating), where the linear segment is
  second order;
* exactness for a source linear in optical depth, at every depth;
* an isothermal box gives I = B; without downwind lines the sweep equals the
  linear one; a step in S never overshoots (the control value is kept between
  the end values).
"""

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("x", [1e-9, 1e-4, 0.03, 0.5, 0.999, 1.0, 1.5, 7.0, 60.0, 700.0])
def test_bezier_weights_closed_forms_and_integrals(x):
    mp.mp.dps = 50
    E, a, b, c = oracle.bezier_weights(x)
    X = mp.mpf(x)
    e = mp.e ** (-X)
    A = (2 - e * (X ** 2 + 2 * X + 2)) / X ** 2
    Bv = 1 - 2 * (e + X - 1) / X ** 2
    C = 2 * (X - 2 + e * (X + 2)) / X ** 2
    for got, want in ((a, A), (b, Bv), (c, C)):
        assert abs(got - float(want)) <= 1e-15 * float(want) + 1e-300
    if x <= 60.0:
        s = lambda t: t / X  # noqa: E731
        k = lambda t: mp.e ** (-(X - t))  # noqa: E731
        for got, basis in ((a, lambda t: (1 - s(t)) ** 2), (b, lambda t: s(t) ** 2),
                           (c, lambda t: 2 * s(t) * (1 - s(t)))):
            want = mp.quad(lambda t: basis(t) * k(t), [0, X])
            assert abs(got - float(want)) <= 1e-15 * float(want)
    Ev, pu, p0 = oracle.psi(x)
    assert abs((a + b + c) - (-np.expm1(-x))) <= 2e-16 * max(1.0, -np.expm1(-x))
    assert abs(a + 0.5 * c - pu) <= 1e-15 * max(pu, 1e-300) + 1e-300
    assert abs(b + 0.5 * c - p0) <= 1e-15 * p0 + 1e-300


def _chain(N, Sfun, kind, T=12.0, nx=2):
    """Emergent intensity at mu = 1 of vertical chains with constant opacity and
    optical depth T over the height, S = Sfun(tau), I_bottom = S at the bottom."""
    z = np.linspace(0.0, 1.0, N)
    g = synth.lattice_grid(nx, 2, z)
    dirs, w = np.array([[0.0, 0.0, 1.0]]), np.array([1.0])
    sel = oracle.select(g, dirs)
    tau = T * (1.0 - g.xyz[:, 2])
    S = Sfun(tau)[:, None]
    chi = np.full_like(S, T)
    if kind == "linear":
        _, I = oracle.fs_voronoi(g, dirs, w, sel, chi, S, S, keep_I=True)
    else:
        _, I = oracle.fs_voronoi_bezier(g, dirs, w, sel, oracle.select_downwind(g, dirs), chi, S, S, keep_I=True)
    return g, tau, I[0, :, 0]


@pytest.mark.parametrize("name", ["quadratic", "exponential", "oscillating"])
def test_third_order_on_vertical_chains(name):
    mp.mp.dps = 30
    Sf, Sm = {
        "quadratic": (lambda t: 1 + t + 0.2 * t ** 2, lambda t: 1 + t + 0.2 * t ** 2),
        "exponential": (lambda t: np.exp(0.3 * t), lambda t: mp.e ** (0.3 * t)),
        "oscillating": (lambda t: 2 + np.sin(t), lambda t: 2 + mp.sin(t)),
    }[name]
    T = 12.0
    exact = float(Sm(T) * mp.e ** (-T) + mp.quad(lambda t: Sm(t) * mp.e ** (-t), [0, T]))
    err = {}
    for kind in ("linear", "bezier"):
        for N in (50, 100, 200):
            g, tau, I = _chain(N, Sf, kind, T)
            top = g.xyz[:, 2] == 1.0
            err[kind, N] = abs(I[top][0] - exact) / exact
    order_b = np.log2(err["bezier", 100] / err["bezier", 200])
    order_l = np.log2(err["linear", 100] / err["linear", 200])
    assert 2.8 < order_b < 3.3, order_b
    assert 1.9 < order_l < 2.2, order_l
    assert err["bezier", 200] < 5e-6 and err["bezier", 200] < err["linear", 200] / 10


def test_linear_source_exact_at_every_depth():
    T, a, b = 7.0, 1.7, 0.45
    g, tau, I = _chain(31, lambda t: a + b * t, "bezier", T, nx=3)
    dt = T - tau
    exact = (a + b * T) * np.exp(-dt) + a * (1 - np.exp(-dt)) + b * (tau + 1 - (T + 1) * np.exp(-dt))
    assert np.max(np.abs(I - exact) / exact) < 1e-12


@pytest.fixture(scope="module")
def recipe():
    atm = synth.make_atmosphere(2000, seed=21)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    return atm, g, dirs, w, oracle.select(g, dirs), oracle.select_downwind(g, dirs)


def test_isothermal_and_no_downwind_lines(recipe):
    atm, g, dirs, w, sel, down = recipe
    rng = np.random.default_rng(0)
    nl = 3
    chi = 10.0 ** rng.uniform(-8, -3, size=(g.n, nl))
    B = np.broadcast_to(np.array([2.5, 7.0, 31.0]), (g.n, nl)).copy()
    J, I = oracle.fs_voronoi_bezier(g, dirs, w, sel, down, chi, B, B, I_top=B, keep_I=True)
    assert np.max(np.abs(I - B[None]) / B[None]) < 1e-14
    # without downwind lines every control value is the midpoint: the linear sweep
    S = rng.uniform(0.5, 2.0, (g.n, nl))
    none = oracle.Selection(np.full_like(down.k1, -1), np.full_like(down.k2, -1), down.w1, down.ds1, down.ds2, 0)
    Jb = oracle.fs_voronoi_bezier(g, dirs, w, sel, none, chi, S, S)
    Jl = oracle.fs_voronoi(g, dirs, w, sel, chi, S, S)
    assert np.max(np.abs(Jb - Jl) / Jl) < 1e-13
    # with them the result differs from the linear sweep
    assert np.max(np.abs(oracle.fs_voronoi_bezier(g, dirs, w, sel, down, chi, S, S) - Jl) / Jl) > 1e-6


def test_step_source_does_not_overshoot():
    """A jump in S along vertical chains: every intensity stays between the
    smallest and largest source value (the boundary takes S there)."""
    N = 60
    z = np.linspace(0.0, 1.0, N)
    g = synth.lattice_grid(2, 2, z)
    dirs, w = np.array([[0.0, 0.0, 1.0]]), np.array([1.0])
    S = np.where(g.xyz[:, 2] < 0.5, 1.0, 5.0)[:, None] * np.array([1.0, 1.0])
    chi = np.array([3.0, 300.0]) * np.ones_like(S)
    _, I = oracle.fs_voronoi_bezier(g, dirs, w, oracle.select(g, dirs), oracle.select_downwind(g, dirs), chi, S,
                                    S, keep_I=True)
    assert I.min() >= 1.0 - 1e-12 and I.max() <= 5.0 + 1e-12


@pytest.mark.parametrize("case", ["clamped", "extremum", "monotone"])
def test_control_value_on_a_three_point_chain(case):
    """Vertical chains of three sites u (bottom), 0, d, opacity 1, I_bottom = 0.
    The middle intensity is alpha S_u + beta S_0 + gamma C with, for
    S = (0, 1, S_d): a steep rise just above 0 (S_d = 101 at 0.01 above)
    pushes the Fritsch-Butland slope to 3 d_u and C = -1/2 below S_u, which
    the clamp returns to S_u = 0; a turn (S_d = 0) gives slope 0 and C = S_0;
    a gentle rise gives the harmonic-mean slope in closed form."""
    zd, Sd = {"clamped": (1.01, 101.0), "extremum": (2.0, 0.0), "monotone": (3.0, 3.0)}[case]
    z = np.array([0.0, 1.0, zd])
    g = synth.lattice_grid(2, 2, z)
    dirs, w = np.array([[0.0, 0.0, 1.0]]), np.array([1.0])
    S = np.array([0.0, 1.0, Sd])[np.searchsorted(z, g.xyz[:, 2])][:, None]
    chi = np.ones_like(S)
    _, I = oracle.fs_voronoi_bezier(g, dirs, w, oracle.select(g, dirs), oracle.select_downwind(g, dirs), chi, S,
                                    np.zeros_like(S), keep_I=True)
    mid = g.xyz[:, 2] == 1.0
    E, a, b, c = oracle.bezier_weights(1.0)
    if case == "clamped":
        C = 0.0
    elif case == "extremum":
        C = 1.0
    else:
        du, xd = 1.0, zd - 1.0
        dd = (Sd - 1.0) / xd
        al = (1.0 + xd / (1.0 + xd)) / 3.0
        C = 1.0 - 0.5 * du * dd / (al * dd + (1.0 - al) * du)
    assert np.allclose(I[0, mid, 0], b * 1.0 + c * C, rtol=1e-14, atol=0)
