"""Reverse (adjoint) sweep of the oracle and the LTE chain rule.

Pins: complex-step derivatives (step 1e-30 i, no cancellation) of a separate
complex-arithmetic forward sweep written here from Eq. 2/5 on a tiny grid,
for every entry of chi, S and I_bottom, and of the full emergent-intensity
misfit L(T, rho) through a complex Planck function; a dot-product identity;
and central finite differences where the perturbation is resolvable in FP64.
"""

import cmath

import numpy as np
import pytest

import synth


def _psi_c(x):
    """e^-x, Psi_u, Psi_0 for complex x (series below |x| = 1/2, closed form above)."""
    if abs(x) < 0.5:
        p0 = 0j
        pu = 0j
        term = x / 2
        for k in range(1, 40):
            p0 += term
            pu += k * term
            term *= -x / (k + 2)
        return cmath.exp(-x), pu, p0
    E = cmath.exp(-x)
    r = (1 - E) / x
    return E, r - E, 1 - r


def _forward_c(g, dirs, sel, chi, S, Ib, It=None):
    """Complex forward intensities [R, n, nl] (top boundary 0 unless It)."""
    R = len(dirs)
    n, nl = chi.shape
    I = np.zeros((R, n, nl), complex)
    for r in range(R):
        sig = 1 if dirs[r, 2] > 0 else -1
        order = sorted(range(n), key=lambda i: (sig * g.xyz[i, 2], i))
        for i in order:
            a, b = sel.k1[r, i], sel.k2[r, i]
            if a < 0:
                I[r, i] = Ib[i] if sig > 0 else (0 if It is None else It[i])
                continue
            for l in range(nl):
                E, pu, p0 = _psi_c(0.5 * (chi[a, l] + chi[i, l]) * sel.ds1[r, i])
                v = E * I[r, a, l] + pu * S[a, l] + p0 * S[i, l]
                if b >= 0:
                    E, pu, p0 = _psi_c(0.5 * (chi[b, l] + chi[i, l]) * sel.ds2[r, i])
                    v2 = E * I[r, b, l] + pu * S[b, l] + p0 * S[i, l]
                    v = sel.w1[r, i] * v + (1 - sel.w1[r, i]) * v2
                I[r, i, l] = v
    return I


@pytest.fixture(scope="module")
def tiny():
    atm = synth.make_atmosphere(45, seed=123)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature(n_mu=1, n_phi=2)
    rng = np.random.default_rng(7)
    nl = 2
    chi = 10 ** rng.uniform(-7.0, -5.0, (g.n, nl))
    S = rng.uniform(1.0, 3.0, (g.n, nl))
    Ib = rng.uniform(2.0, 4.0, (g.n, nl))
    # a fixed random linear functional of all intensities and of J
    cI = rng.standard_normal((len(dirs), g.n, nl))
    cJ = rng.standard_normal((g.n, nl))
    return g, dirs, w, chi, S, Ib, cI, cJ


def _L_c(tiny, sel, chi, S, Ib):
    g, dirs, w, _, _, _, cI, cJ = tiny
    I = _forward_c(g, dirs, sel, chi, S, Ib)
    J = np.tensordot(w, I, axes=(0, 0))
    return np.sum(cI * I) + np.sum(cJ * J)


def test_reverse_sweep_matches_complex_step(orc, tiny):
    g, dirs, w, chi, S, Ib, cI, cJ = tiny
    sel = orc.select(g, dirs)
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, keep_I=True)
    gc, gS, gIb, gIt = orc.fs_voronoi_vjp(g, dirs, w, sel, chi, S, I, dL_dI=cI, dL_dJ=cJ)
    h = 1e-30
    for name, base, grad in (("S", S, gS), ("Ib", Ib, gIb)):
        for q in range(base.size):
            pert = base.astype(complex).copy()
            pert.flat[q] += 1j * h
            args = {"chi": chi.astype(complex), "S": S.astype(complex), "Ib": Ib.astype(complex)}
            args[name] = pert
            d = _L_c(tiny, sel, args["chi"], args["S"], args["Ib"]).imag / h
            assert abs(grad.flat[q] - d) <= 1e-12 * max(1.0, abs(d)), (name, q, d, grad.flat[q])
    # the seeds of downward-ray boundary sites land in dL/dI_top
    assert np.all(np.isfinite(gIt)) and np.any(gIt != 0)


def test_reverse_sweep_relative_accuracy_on_chi(orc, tiny):
    """chi derivatives are large (x = chi * ds with ds ~ 1e6 m): check them relatively."""
    g, dirs, w, chi, S, Ib, cI, cJ = tiny
    sel = orc.select(g, dirs)
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, keep_I=True)
    gc, _, _, _ = orc.fs_voronoi_vjp(g, dirs, w, sel, chi, S, I, dL_dI=cI, dL_dJ=cJ)
    h = 1e-30
    worst = 0.0
    scale = np.max(np.abs(gc))
    for q in range(chi.size):
        pert = chi.astype(complex).copy()
        step = h * chi.flat[q]
        pert.flat[q] += 1j * step
        d = _L_c(tiny, sel, pert, S.astype(complex), Ib.astype(complex)).imag / step
        worst = max(worst, abs(gc.flat[q] - d) / scale)
    assert worst <= 1e-12


def test_dot_product_identity(orc, tiny):
    """<dL/dS, dS> equals the directional derivative of L along dS (L is linear in S and I_bottom)."""
    g, dirs, w, chi, S, Ib, cI, cJ = tiny
    sel = orc.select(g, dirs)
    J, I = orc.fs_voronoi(g, dirs, w, sel, chi, S, Ib, keep_I=True)
    _, gS, gIb, _ = orc.fs_voronoi_vjp(g, dirs, w, sel, chi, S, I, dL_dI=cI, dL_dJ=cJ)
    rng = np.random.default_rng(9)
    dS = rng.standard_normal(S.shape)
    dIb = rng.standard_normal(Ib.shape)
    J2, I2 = orc.fs_voronoi(g, dirs, w, sel, chi, dS, dIb, keep_I=True)
    lhs = np.sum(gS * dS) + np.sum(gIb * dIb)
    rhs = np.sum(cI * I2) + np.sum(cJ * J2)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


_H, _C, _K = 6.62607015e-34, 299792458.0, 1.380649e-23


def _lte_c(lam, kappa0, T, rho):
    """Complex grey LTE continuum (chi = kappa0 rho^2 T^9, S = B_lambda(T) in kW m^-2 nm^-1 sr^-1)."""
    chi = np.stack([kappa0 * rho * rho * T**9 for _ in lam], axis=1)
    S = np.stack([2 * _H * _C * _C / l**5 / (np.exp(_H * _C / (l * _K * T)) - 1) * 1e-12 for l in lam], axis=1)
    return chi, S


@pytest.fixture(scope="module")
def small_lte():
    atm = synth.make_atmosphere(70, seed=31)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature(n_mu=2, n_phi=2)
    lam = np.array([500e-9, 650e-9])
    Tt = atm.T * (1 + 0.02 * np.random.default_rng(1).standard_normal(g.n))
    return atm, g, dirs, w, lam, Tt


def _misfit_c(g, dirs, sel, lam, kappa0, T, rho, target, em):
    chi, S = _lte_c(lam, kappa0, T, rho)
    I = _forward_c(g, dirs, sel, chi, S, S)
    L = 0j
    for r in range(len(dirs)):
        if dirs[r, 2] > 0:
            d = I[r, em[r]] - target[r]
            L += np.sum(d * d)
    return L


def test_temperature_density_gradient_matches_complex_step(orc, small_lte):
    atm, g, dirs, w, lam, Tt = small_lte
    sel = orc.select(g, dirs)
    _, _, _, It = orc.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, Tt, atm.rho)
    em = orc.emergent_sites(g, dirs)
    target = {r: It[r, em[r]] for r in range(len(dirs)) if dirs[r, 2] > 0}
    L, gT, gr, _ = orc.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, atm.T, atm.rho, target)
    h = 1e-30
    for arr, grad in ((atm.T, gT), (atm.rho, gr)):
        scale = np.max(np.abs(grad))
        for i in range(g.n):
            a = arr.astype(complex).copy()
            a[i] += 1j * h * arr[i]
            T = a if arr is atm.T else atm.T.astype(complex)
            rho = a if arr is atm.rho else atm.rho.astype(complex)
            d = _misfit_c(g, dirs, sel, lam, atm.kappa0, T, rho, target, em).imag / (h * arr[i])
            assert abs(d - grad[i]) <= 1e-11 * scale, (i, d, grad[i])


def test_gradient_matches_central_differences_where_resolvable(orc):
    """Central differences (relative step 1e-5) agree where the perturbed site is
    optically thick enough for the change of L to stand well above rounding."""
    atm = synth.make_atmosphere(400, seed=31)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    dirs, w = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    lam = np.array([500e-9, 650e-9])
    Tt = atm.T * (1 + 0.02 * np.random.default_rng(1).standard_normal(g.n))
    _, _, _, It = orc.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, Tt, atm.rho)
    em = orc.emergent_sites(g, dirs)
    target = {r: It[r, em[r]] for r in range(len(dirs)) if dirs[r, 2] > 0}
    L, gT, gr, _ = orc.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, atm.T, atm.rho, target)
    chi, _ = orc.lte(lam, atm.kappa0, atm.T, atm.rho)
    thick = np.nonzero(chi[:, 0] * 3e5 > 1e-2)[0]
    picks = np.random.default_rng(2).choice(thick, 10, replace=False)
    for i in picks:
        for which, grad in (("T", gT), ("rho", gr)):
            base = atm.T if which == "T" else atm.rho
            h = 1e-5 * base[i]
            vals = []
            for sgn in (1, -1):
                a = base.copy()
                a[i] += sgn * h
                T, rho = (a, atm.rho) if which == "T" else (atm.T, a)
                vals.append(orc.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, T, rho, target)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-4 * abs(grad[i]) + 1e-9 * abs(L) / base[i], (which, i, fd, grad[i])
