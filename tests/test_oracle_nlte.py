"""Two-level Lambda iteration (Sect. 2.1 Eq. 3-4; stop rule near 1e-3, Sect. 3.3).

Pins: the iteration's fixed point equals a dense linear solve of the same
discrete problem; an isothermal thermalised box has S_L = B as an exact fixed
point; resuming from a saved S_L reproduces an uninterrupted run bitwise; and
the surface value of a semi-infinite constant-property atmosphere approaches
sqrt(eps) B (the exact two-stream result S(0) = sqrt(eps) B, which holds here
because every ray on a lattice column is carried along vertical lines) with
second-order convergence in the log-tau spacing.
"""

import numpy as np
import pytest

import synth
from oracle import nlte


@pytest.fixture(scope="module")
def small():
    atm = synth.make_atmosphere(300, seed=31)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    return atm, g, dirs, w


def _line(g, nl, seed):
    rng = np.random.default_rng(seed)
    x = np.linspace(-3, 3, nl)
    wl = np.full(nl, x[1] - x[0])
    wl[0] *= 0.5
    wl[-1] *= 0.5
    width = rng.uniform(0.8, 1.2, g.n)
    phi = np.exp(-(x[None, :] / width[:, None]) ** 2)
    phi /= np.sum(wl[None, :] * phi, axis=1)[:, None]
    return phi, wl


def test_lambda_iteration_reaches_dense_fixed_point(orc, small):
    atm, g, dirs, w = small
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(1)
    phi, wl = _line(g, 5, 2)
    chi_c = 10 ** rng.uniform(-7, -6, g.n)
    chi_L = 10 ** rng.uniform(-6, -5, g.n)
    B = rng.uniform(1.0, 3.0, g.n)
    eps = 1e-2
    S_it, hist, nit, ok = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps,
                                              max_iter=3000, tol=1e-13)
    assert ok
    S_dense = nlte.dense_fixed_point(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps)
    assert np.max(np.abs(S_it - S_dense) / S_dense) < 1e-10


def test_isothermal_fixed_point(orc, small):
    atm, g, dirs, w = small
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(3)
    phi, wl = _line(g, 7, 4)
    chi_c = 10 ** rng.uniform(-8, -5, g.n)
    chi_L = 10 ** rng.uniform(-6, -4, g.n)
    B = np.full(g.n, 2.75)
    S1, dS = nlte.lambda_step(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, 1e-3, B.copy(), I_top=B)
    assert dS < 1e-14
    assert np.max(np.abs(S1 - 2.75)) < 1e-14 * 2.75 * 10


def test_resume_is_bitwise(orc, small):
    atm, g, dirs, w = small
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(5)
    phi, wl = _line(g, 3, 6)
    chi_c = 10 ** rng.uniform(-7, -6, g.n)
    chi_L = 10 ** rng.uniform(-6, -5, g.n)
    B = rng.uniform(1.0, 3.0, g.n)
    a, _, _, _ = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, 1e-2, max_iter=10, tol=0)
    b, _, _, _ = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, 1e-2, max_iter=4, tol=0)
    b, _, _, _ = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, 1e-2, max_iter=6, tol=0,
                                     S_start=b)
    assert np.array_equal(a, b)


def _sqrt_eps_column(orc, eps, ppd):
    """Surface S_L / (sqrt(eps) B) of a monochromatic, constant-property column."""
    tau_max = 1e3 / np.sqrt(eps)
    ndec = np.log10(tau_max) + 6
    taus = np.r_[0.0, np.logspace(-6, np.log10(tau_max), int(round(ndec * ppd)) + 1)]
    z = (tau_max - taus)[::-1]           # chi = 1 so z measures optical depth from the top
    g = synth.lattice_grid(2, 2, z)
    dirs, w = synth.vertical_quadrature()
    sel = orc.select(g, dirs)
    n = g.n
    phi = np.ones((n, 1))
    wl = np.ones(1)
    B = np.ones(n)
    groups = [np.arange(4 * k, 4 * k + 4) for k in range(len(z))]
    S = nlte.dense_fixed_point(g, dirs, w, sel, np.zeros(n), np.ones(n), phi, wl, B, eps, groups=groups)
    return S[-1] / np.sqrt(eps)


def test_sqrt_eps_law_eps_1e2(orc):
    vals = [_sqrt_eps_column(orc, 1e-2, p) for p in (5, 10, 20, 40)]
    errs = np.abs(1.0 - np.array(vals))
    assert np.all(np.diff(errs) < 0)
    assert np.all(errs[:-1] / errs[1:] > 2.5)
    assert errs[-1] < 0.02


@pytest.mark.slow
def test_sqrt_eps_law_eps_1e4(orc):
    vals = [_sqrt_eps_column(orc, 1e-4, p) for p in (40, 80, 160)]
    errs = np.abs(1.0 - np.array(vals))
    assert np.all(np.diff(errs) < 0)
    assert np.all(errs[:-1] / errs[1:] > 2.0)
    assert errs[-1] < 0.05


def test_lambda_diag_is_the_diagonal_of_lambda(orc, small):
    """dJ_i/dS_i by brute force: the formal solution of a unit source at one site
    (no boundary radiation) has J_i = Lambda_ii at that site."""
    atm, g, dirs, w = small
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(11)
    nl = 3
    chi = 10 ** rng.uniform(-7.0, -4.0, (g.n, nl))
    Ld = orc.lambda_diag(g, dirs, w, sel, chi)
    zero = np.zeros((g.n, nl))
    for i in rng.choice(g.n, 40, replace=False):
        S = zero.copy()
        S[i] = 1.0
        J = orc.fs_voronoi(g, dirs, w, sel, chi, S, zero)
        assert np.allclose(J[i], Ld[i], rtol=1e-13, atol=0), (i, J[i], Ld[i])
    # boundary sites of every ray contribute nothing, interior ones are in (0, 1)
    assert np.all(Ld >= 0) and np.all(Ld < 1)


def test_line_diag_is_the_diagonal_of_the_jbar_map(orc):
    atm = synth.make_atmosphere(60, seed=8)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(12)
    phi, wl = _line(g, 7, 13)
    chi_c = 10 ** rng.uniform(-7, -6, g.n)
    chi_L = 10 ** rng.uniform(-6, -5, g.n)
    B = rng.uniform(1.0, 3.0, g.n)
    M, _, _ = nlte.jbar_matrix(g, dirs, w, sel, chi_c, chi_L, phi, wl, B)
    Lbar = nlte.line_diag(g, dirs, w, sel, chi_c, chi_L, phi, wl)
    assert np.max(np.abs(np.diag(M) - Lbar)) <= 1e-13 * np.max(np.abs(Lbar))


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_accelerated_iteration_reaches_dense_fixed_point(orc, small, eps):
    """The Jacobi-accelerated iteration has the same fixed point and gets there
    in fewer iterations than the plain one."""
    atm, g, dirs, w = small
    sel = orc.select(g, dirs)
    rng = np.random.default_rng(1)
    phi, wl = _line(g, 5, 2)
    chi_c = 10 ** rng.uniform(-7, -6, g.n)
    chi_L = 10 ** rng.uniform(-5, -4, g.n)
    B = rng.uniform(1.0, 3.0, g.n)
    S_dense = nlte.dense_fixed_point(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps)
    S_a, hist_a, nit_a, ok_a = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps, max_iter=3000,
                                                   tol=1e-12, accel=True)
    assert ok_a
    assert np.max(np.abs(S_a - S_dense) / S_dense) < 1e-9
    _, _, nit_p, _ = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps, max_iter=3000, tol=1e-6)
    _, _, nit_a6, _ = nlte.lambda_iterate(g, dirs, w, sel, chi_c, chi_L, phi, wl, B, eps, max_iter=3000, tol=1e-6,
                                          accel=True)
    assert nit_a6 < nit_p
