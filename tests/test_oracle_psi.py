"""Segment weights of the linear-source formal solution (Sect. 2.1 Eq. 2 with S linear, Sect. 2.5).

Pins: the exact integrals evaluated in 50-digit arithmetic (mpmath), the exact
result for constant and linear S on one segment, and the identity
Psi_u + Psi_0 = 1 - e^-x (the weights of a constant source).
"""

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 50

XS = sorted(set([0.0, 1e-300, 1e-200, 1e-30, 1e-16, 1e-12, 1e-8, 1e-5, 1e-3, 0.01, 0.1, 0.3, 0.4999999,
                 0.5, 0.5000001, 0.7, 1.0, 2.0, 5.0, 10.0, 30.0, 100.0, 700.0, 800.0, 1000.0]
                + list(np.logspace(-300, 3, 61))))


def _exact(x):
    """Closed-form weights at a working precision large enough that x - (1 - e^-x)
    keeps 50 significant digits (about 2*|log10 x| extra digits for tiny x)."""
    if x == 0:
        return mp.mpf(1), mp.mpf(0), mp.mpf(0)
    extra = int(2 * max(0.0, -np.log10(float(x)))) + 10
    with mp.workdps(50 + extra):
        xm = mp.mpf(x)
        E = mp.exp(-xm)
        e0 = -mp.expm1(-xm)
        e1 = xm - e0
        return +E, e0 - e1 / xm, e1 / xm


def _rel(a, b):
    b = float(b)
    if b == 0.0:
        return abs(a)
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("x", XS)
def test_psi_against_50_digit_integrals(orc, x):
    E, pu, p0 = orc.psi(x)
    Ee, pue, p0e = _exact(x)
    assert _rel(E, Ee) <= 2e-16 or abs(E - float(Ee)) < 1e-300
    assert _rel(pu, pue) <= 1e-14
    assert _rel(p0, p0e) <= 1e-14


@pytest.mark.parametrize("x", [1e-9, 1e-4, 0.2, 0.49, 0.51, 1.5, 20.0])
def test_psi_integral_definition(orc, x):
    # Psi_u = int_0^x (1 - t/x) e^-(x-t) dt, Psi_0 = int_0^x (t/x) e^-(x-t) dt
    xm = mp.mpf(x)
    pu_e = mp.quad(lambda t: (1 - t / xm) * mp.exp(-(xm - t)), [0, xm])
    p0_e = mp.quad(lambda t: (t / xm) * mp.exp(-(xm - t)), [0, xm])
    _, pu, p0 = orc.psi(x)
    assert _rel(pu, pu_e) <= 1e-14
    assert _rel(p0, p0_e) <= 1e-14


@pytest.mark.parametrize("x", [1e-12, 1e-6, 0.05, 0.3, 0.5, 0.8, 3.0, 50.0])
def test_dpsi_against_derivative(orc, x):
    xm = mp.mpf(x)
    h = xm * mp.mpf("1e-18")
    du_e = mp.diff(lambda t: _exact(t)[1], xm, h=h)
    d0_e = mp.diff(lambda t: _exact(t)[2], xm, h=h)
    du, d0 = orc.dpsi(x)
    assert _rel(du, du_e) <= 1e-13
    assert _rel(d0, d0_e) <= 1e-13


def test_dpsi_at_zero(orc):
    du, d0 = orc.dpsi(0.0)
    assert du == 0.5 and d0 == 0.5


def test_constant_source_identity(orc):
    for x in XS:
        E, pu, p0 = orc.psi(x)
        assert abs((pu + p0) - (1.0 - E)) <= 4e-16 * max(1.0, 1.0 - E) + 1e-300


def test_one_segment_linear_source_exact(orc):
    # dI/dt = S - I with S(t) = a + b t along t in [0, x], I(0) = I0
    for x in [1e-7, 0.3, 0.5, 2.0, 40.0]:
        a, b, I0 = 1.3, 0.7, 2.9
        xm = mp.mpf(x)
        exact = I0 * mp.exp(-xm) + mp.quad(lambda t: (a + b * t) * mp.exp(-(xm - t)), [0, xm])
        E, pu, p0 = orc.psi(x)
        got = E * I0 + pu * a + p0 * (a + b * x)
        assert _rel(got, exact) <= 1e-14
