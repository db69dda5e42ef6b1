"""Inputs of the two-level line problem (Sect. 2.1 Eq. 3, Sect. 2.2).

The paper's atom (Table 1, Johnson rates, Transparency.jl opacities) cannot be
rebuilt here; a single line with a photon-destruction probability eps stands
in for it:

* line centre lambda0 = 121.568 nm (the paper's Lyman-alpha-like line);
* Doppler width per site dl_D = (lambda0 / c) sqrt(2 k T / m_H + xi^2) with
  xi = 2 km/s microturbulence;
* n_lambda points uniform over lambda0 +- 5 dl_D(6500 K);
* Voigt profile with damping a = 0.01, phi = H(a, v) / (sqrt(pi) dl_D) per nm,
  renormalised per site so that sum_lambda w_lambda phi = 1 with trapezoid
  weights w_lambda (in nm), which keeps S_L = B an exact fixed point of an
  isothermal box;
* line opacity chi_L phi_lambda with chi_L = K_L rho, K_L set so that the
  line-centre optical depth of the unperturbed stratification reaches 1 at
  z = 1.5 Mm (above 0.5 Mm T0 = 4200 K and rho decays exponentially, so the
  integral to infinity is closed-form).

The profile is input data (like the quadrature); the method's arithmetic, the
opacity and source assembly and the Lambda iteration, lives in the oracle and
the HIP library.
"""

from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np
from scipy.special import voigt_profile

from .atmosphere import H_RHO, MM, T0_of_z, rho_of_z

LAMBDA0_NM = 121.568
C_LIGHT = 299792458.0
K_BOLTZMANN = 1.380649e-23
M_H = 1.6735575e-27  # kg, hydrogen atom
XI_MICRO = 2.0e3     # m/s
_ROWS = 65536        # sites per block of the profile table


def doppler_width_nm(T, lam0_nm=LAMBDA0_NM, xi=XI_MICRO):
    T = np.asarray(T, dtype=np.float64)
    return lam0_nm / C_LIGHT * np.sqrt(2.0 * K_BOLTZMANN * T / M_H + xi * xi)


@dataclass
class LineSetup:
    lam_nm: np.ndarray   # [nl] wavelengths (nm)
    wlam: np.ndarray     # [nl] trapezoid weights (nm)
    phi: np.ndarray      # [n, nl] profile per nm, sum_l wlam phi = 1 per site
    chi_line: np.ndarray  # [n] line opacity scale K_L rho (m^-1 nm)
    K_L: float
    damping: float


def line_setup(T, rho, n_lambda: int = 101, damping: float = 0.01, half_width: float = 5.0,
               workers: int = 1) -> LineSetup:
    """Line data of every site; `workers` threads fill row blocks of phi (the
    result does not depend on it)."""
    T = np.asarray(T, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    dl_ref = float(doppler_width_nm(6500.0))
    lam = LAMBDA0_NM + np.linspace(-half_width, half_width, n_lambda) * dl_ref
    wl = np.full(n_lambda, lam[1] - lam[0] if n_lambda > 1 else 1.0)
    if n_lambda > 1:
        wl[0] *= 0.5
        wl[-1] *= 0.5
    dl = doppler_width_nm(T)
    phi = np.empty((len(T), n_lambda), np.float64)

    def rows(a):
        b = min(a + _ROWS, len(T))
        # H(a, v)/(sqrt(pi) dl) is the normalised Voigt profile with Gaussian sigma = dl/sqrt(2), Lorentz gamma = a dl
        p = voigt_profile((lam[None, :] - LAMBDA0_NM), dl[a:b, None] / np.sqrt(2.0), damping * dl[a:b, None])
        phi[a:b] = p / np.sum(wl[None, :] * p, axis=1)[:, None]

    starts = range(0, len(T), _ROWS)
    if workers > 1:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(rows, starts))
    else:
        for a in starts:
            rows(a)
    # line-centre tau = 1 at 1.5 Mm on the unperturbed stratification
    T_top = float(T0_of_z(1.5 * MM))
    dlt = float(doppler_width_nm(T_top))
    phi0 = float(voigt_profile(0.0, dlt / np.sqrt(2.0), damping * dlt))
    K_L = 1.0 / (phi0 * float(rho_of_z(1.5 * MM)) * H_RHO)
    return LineSetup(lam_nm=lam, wlam=wl, phi=np.ascontiguousarray(phi), chi_line=K_L * rho, K_L=K_L,
                     damping=damping)


def line_case(job):
    """One seeded atmosphere of the two-level workloads with its Voronoi grid and
    line data: job = (n_sites, seed) -> (Atmosphere, VoronoiGrid, LineSetup with
    101 wavelengths). A module-level function, so a process pool can build the
    atmospheres of a batch in parallel."""
    from .atmosphere import make_atmosphere
    from .voronoi import voronoi_neighbours

    n, seed = job
    atm = make_atmosphere(n, seed=seed)
    g = voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    return atm, g, line_setup(atm.T, atm.rho, n_lambda=101)
