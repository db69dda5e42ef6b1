"""Site-sampling densities of the grid-design study (Sect. 2.4) and the
searchlight-beam set-up (Sect. 3.1).

The paper places the sites by rejection sampling (Sect. 2.4, four steps) from a
target density f(r) that is large where the radiation forms. Besides the
recipe's own |d ln tau / dz| (``sample_sites``), three targets it names are
evaluated here from the synthetic temperature and density (readings of the
paper, which gives no units or constants for them):

* ``alpha_c``  the continuum extinction, whose shape is rho^2 T^9 in the grey
  recipe (the normalising constant does not matter to rejection sampling);
* ``log_nhii`` log10 of the LTE proton density n_p [m^-3] of pure hydrogen
  from the Saha equation, n_p^2 / (N_H - n_p) = (2 pi m_e k T / h^2)^(3/2)
  exp(-13.598 eV / k T), with N_H = rho / (1.4 m_H) (helium by mass);
* ``log_nh_t`` (log10 N_H)^-2 T^-2/5 with N_H in m^-3.

These only decide where sites go; no value computed here enters the formal
solution.
"""

from __future__ import annotations

import numpy as np

from .atmosphere import BoxSpec, T0_of_z, horizontal_field, locality_order, rho_of_z, sample_field

M_H = 1.6735575e-27     # kg
M_E = 9.1093837015e-31  # kg
K_B = 1.380649e-23      # J / K
H_PLANCK = 6.62607015e-34
CHI_H = 13.598434 * 1.602176634e-19  # J
MEAN_MASS = 1.4  # mass per hydrogen atom in units of m_H (helium by mass)

DENSITIES = ("alpha_c", "log_nhii", "log_nh_t")


def _state(xyz, box, field_seed, temp_perturbation=0.05):
    d = sample_field(horizontal_field(field_seed, box), xyz[:, 0], xyz[:, 1], box)
    T = T0_of_z(xyz[:, 2]) * (1.0 + temp_perturbation * d)
    return T, rho_of_z(xyz[:, 2])


def target_density(name: str, xyz, box: BoxSpec = BoxSpec(), field_seed: int = 1041 + 7919):
    """Target density f >= 0 of one of ``DENSITIES`` at positions xyz [m, 3]."""
    xyz = np.asarray(xyz, np.float64)
    T, rho = _state(xyz, box, field_seed)
    n_h = rho / (MEAN_MASS * M_H)
    if name == "alpha_c":
        return rho ** 2 * T ** 9
    if name == "log_nhii":
        phi = (2.0 * np.pi * M_E * K_B * T / H_PLANCK ** 2) ** 1.5 * np.exp(-CHI_H / (K_B * T))
        n_p = 0.5 * (-phi + np.sqrt(phi * phi + 4.0 * phi * n_h))
        return np.maximum(np.log10(np.maximum(n_p, 1.0)), 0.0)
    if name == "log_nh_t":
        return np.log10(n_h) ** -2 * T ** -0.4
    raise ValueError(f"unknown density {name!r}")


def sample_sites_density(n: int, seed: int, name: str, box: BoxSpec = BoxSpec(), field_seed: int = 1041 + 7919,
                         batch: int = 1 << 20):
    """Rejection-sample n sites from ``target_density(name)`` (Sect. 2.4): propose
    uniformly, draw the rejection level uniformly in [0, f_max), accept when
    f(proposal) >= level. f_max is 1.05 times the largest f over 2^20 seeded
    probe points and the z-axis extremes. Sites are numbered in
    ``locality_order``, as ``sample_sites`` numbers them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(box.lo, np.float64)
    L = box.L
    probe = lo + rng.random((1 << 20, 3)) * L
    zs = np.linspace(box.lo[2], box.hi[2], 4097)
    edge = np.stack([np.full_like(zs, lo[0]), np.full_like(zs, lo[1]), zs], 1)
    fmax = 1.05 * max(target_density(name, probe, box, field_seed).max(),
                      target_density(name, edge, box, field_seed).max())
    out, got = [], 0
    while got < n:
        prop = lo + rng.random((batch, 3)) * L
        acc = prop[target_density(name, prop, box, field_seed) >= rng.random(batch) * fmax]
        out.append(acc)
        got += len(acc)
    xyz = np.concatenate(out)[:n]
    return np.ascontiguousarray(xyz[locality_order(xyz, box)])


def searchlight(n_side: int = 51, seed: int = 1041, radius: float = 0.2, theta_deg: float = 20.0):
    """The searchlight test of Sect. 3.1: a 1 m box with n_side^3 sites drawn
    uniformly (Voronoi) and the regular n_side^3 lattice, one ray inclined by
    theta from the vertical, and a circular beam of unit intensity and the given
    radius centred on the bottom face. Returns (sites [n, 3], box lo, box hi,
    direction [1, 3], weight [1], beam(x, y) -> 0/1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_side ** 3
    xyz = rng.random((n, 3))
    th = np.deg2rad(theta_deg)
    d = np.array([[np.sin(th), 0.0, np.cos(th)]])

    def beam(x, y):
        return (((np.asarray(x) - 0.5) ** 2 + (np.asarray(y) - 0.5) ** 2) <= radius ** 2).astype(np.float64)

    return xyz, np.zeros(3), np.ones(3), d, np.array([1.0]), beam
