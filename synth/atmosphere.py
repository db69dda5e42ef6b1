"""Bifrost-like synthetic stratified atmosphere and rejection-sampled Voronoi sites.

The paper's atmosphere is a Bifrost snapshot (Sect. 2.3) that is not available,
so a seeded analytic stand-in is used (all SI, lengths in metres):

* periodic box 6 x 6 Mm horizontally, z in [-0.5, 2.5] Mm;
* T0(z) = 4200 + 1150 * (1 - tanh((z - 0.25 Mm) / 0.125 Mm)) K, i.e. about
  6500 K at the bottom falling to 4200 K above 0.5 Mm;
* rho(z) = 3e-4 * exp(-z / 150 km) kg m^-3;
* T(x, y, z) = T0(z) * (1 + 0.05 * delta(x, y)), with delta a zero-mean,
  unit-variance Gaussian random field of correlation length 1 Mm;
* the grey opacity normalisation kappa0 is fixed by tau(z=0) = 1 on the
  unperturbed stratification for chi = kappa0 * rho^2 * T^9 (mass absorption
  coefficient kappa0 * rho * T^9 times rho).

Sites are drawn by the four-step rejection sampling of Sect. 2.4 with target
density f(z) = |d ln tau / dz|.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MM = 1.0e6  # one megametre in metres
KM = 1.0e3


@dataclass(frozen=True)
class BoxSpec:
    lo: tuple = (0.0, 0.0, -0.5 * MM)
    hi: tuple = (6.0 * MM, 6.0 * MM, 2.5 * MM)
    periodic_xy: bool = True

    @property
    def L(self):
        return np.asarray(self.hi, dtype=np.float64) - np.asarray(self.lo, dtype=np.float64)


def T0_of_z(z):
    """Unperturbed temperature stratification [K] at height z [m]."""
    z = np.asarray(z, dtype=np.float64)
    return 4200.0 + 1150.0 * (1.0 - np.tanh((z - 0.25 * MM) / (0.125 * MM)))


RHO0 = 3.0e-4          # kg m^-3 at z = 0
H_RHO = 150.0 * KM     # density scale height


def rho_of_z(z):
    """Mass density [kg m^-3] at height z [m]."""
    z = np.asarray(z, dtype=np.float64)
    return RHO0 * np.exp(-z / H_RHO)


def horizontal_field(seed: int, box: BoxSpec = BoxSpec(), n: int = 256, corr_len: float = 1.0 * MM):
    """Periodic Gaussian random field on an n x n grid covering the box's x-y extent.

    White noise is filtered in Fourier space by exp(-k^2 l^2 / 4), which gives
    the correlation function exp(-r^2 / (2 l^2)); the result is shifted and
    scaled to zero mean and unit standard deviation. Returns the [n, n] array
    indexed [ix, iy].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n, n))
    Lx, Ly = box.L[0], box.L[1]
    kx = 2.0 * np.pi * np.fft.fftfreq(n, d=Lx / n)
    ky = 2.0 * np.pi * np.fft.fftfreq(n, d=Ly / n)
    k2 = kx[:, None] ** 2 + ky[None, :] ** 2
    filt = np.exp(-k2 * corr_len**2 / 4.0)
    f = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    f -= f.mean()
    f /= f.std()
    return f


def sample_field(field2d, x, y, box: BoxSpec = BoxSpec()):
    """Periodic bilinear interpolation of a [n, n] grid field (nodes at lo + i*L/n)."""
    n0, n1 = field2d.shape
    fx = (np.asarray(x) - box.lo[0]) / box.L[0] * n0
    fy = (np.asarray(y) - box.lo[1]) / box.L[1] * n1
    i0 = np.floor(fx).astype(np.int64)
    j0 = np.floor(fy).astype(np.int64)
    tx = fx - i0
    ty = fy - j0
    i0 %= n0
    j0 %= n1
    i1 = (i0 + 1) % n0
    j1 = (j0 + 1) % n1
    return ((1 - tx) * (1 - ty) * field2d[i0, j0] + tx * (1 - ty) * field2d[i1, j0]
            + (1 - tx) * ty * field2d[i0, j1] + tx * ty * field2d[i1, j1])


def kappa0_and_density(box: BoxSpec = BoxSpec(), n_z: int = 300001):
    """Grey-opacity normalisation and the site-density profile.

    Integrates tau_unit(z) = int_z^inf rho^2 T0^9 dz' on the unperturbed
    stratification from the top down (reverse cumulative trapezoid), adding
    the analytic exponential tail above the box (T0 is constant there and
    rho^2 decays with scale height H/2). kappa0 = 1 / tau_unit(0).

    Returns (kappa0, z_tab [n_z], f_tab [n_z]) with f = |d ln tau / dz| =
    chi / tau on the table.
    """
    zlo, zhi = box.lo[2], box.hi[2]
    z = np.linspace(zlo, zhi, n_z)
    g = rho_of_z(z) ** 2 * T0_of_z(z) ** 9  # chi / kappa0
    tail = g[-1] * H_RHO / 2.0
    seg = 0.5 * (g[1:] + g[:-1]) * np.diff(z)
    tau = np.empty_like(z)
    tau[-1] = tail
    tau[:-1] = tail + np.cumsum(seg[::-1])[::-1]
    tau0 = np.interp(0.0, z, tau)
    kappa0 = 1.0 / tau0
    f = g / tau  # kappa0 cancels
    return kappa0, z, f


def _spread_bits(v, bits=16):
    """Interleave the low `bits` bits of v with zeros (bit b moves to bit 2b)."""
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(bits):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
    return out


def locality_order(xyz, box: BoxSpec = BoxSpec()):
    """Permutation that numbers sites the way a block-structured container
    visits them: horizontal slabs one mean site spacing thick, bottom to top,
    and inside a slab the Morton (Z-order) curve of (x, y) on a 2^16 x 2^16
    lattice of the box. Sites that are close in space get close numbers, so
    [site][wavelength] rows that one level of a sweep touches lie close
    together in memory. Stable: ties keep the sampling order."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n = len(xyz)
    if n == 0:
        return np.zeros(0, np.int64)
    lo = np.asarray(box.lo, dtype=np.float64)
    L = box.L
    h = float(np.prod(L) / n) ** (1.0 / 3.0)
    slab = np.floor((xyz[:, 2] - lo[2]) / h).astype(np.int64)
    q = np.clip(np.floor((xyz[:, :2] - lo[:2]) / L[:2] * 65536.0), 0, 65535).astype(np.int64)
    morton = _spread_bits(q[:, 0]) | (_spread_bits(q[:, 1]) << np.uint64(1))
    return np.lexsort((morton, slab))


def sample_sites(n: int, seed: int, box: BoxSpec = BoxSpec(), uniform: bool = False, batch: int = 1 << 20,
                 ordered: bool = True):
    """Rejection-sample n sites (Sect. 2.4, four steps).

    1. propose a position uniformly in the box and evaluate the target density
       there; 2. draw a uniform rejection level in [0, f_max); 3. accept if the
       proposal density is at least the rejection level; 4. repeat until n
       sites are accepted. With ``uniform=True`` every proposal is accepted
       (the searchlight test samples sites uniformly). With ``ordered`` (the
       default) the accepted sites are numbered in ``locality_order``;
       otherwise in the order they were accepted.
    Returns float64 [n, 3].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(box.lo, dtype=np.float64)
    L = box.L
    if uniform:
        xyz = lo + rng.random((n, 3)) * L
    else:
        _, zt, ft = kappa0_and_density(box)
        fmax = ft.max()
        out = []
        got = 0
        while got < n:
            prop = lo + rng.random((batch, 3)) * L
            fp = np.interp(prop[:, 2], zt, ft)
            u = rng.random(batch) * fmax
            acc = prop[fp >= u]
            out.append(acc)
            got += len(acc)
        xyz = np.concatenate(out)[:n]
    return np.ascontiguousarray(xyz[locality_order(xyz, box)]) if ordered else xyz


@dataclass
class Atmosphere:
    """Per-site thermodynamic state of a synthetic atmosphere (caller site order)."""

    xyz: np.ndarray          # [n, 3] float64, metres
    T: np.ndarray            # [n] float64, K
    rho: np.ndarray          # [n] float64, kg m^-3
    kappa0: float            # grey normalisation, chi = kappa0 * rho^2 * T^9
    box: BoxSpec = field(default_factory=BoxSpec)
    seed: int = 0


def make_atmosphere(n_sites: int, seed: int = 1041, box: BoxSpec = BoxSpec(), xyz=None,
                    temp_perturbation: float = 0.05, field_seed=None) -> Atmosphere:
    """Sites (rejection-sampled unless ``xyz`` is given) with T and rho from the recipe."""
    if xyz is None:
        xyz = sample_sites(n_sites, seed, box)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    delta = horizontal_field(seed + 7919 if field_seed is None else field_seed, box)
    d = sample_field(delta, xyz[:, 0], xyz[:, 1], box)
    T = T0_of_z(xyz[:, 2]) * (1.0 + temp_perturbation * d)
    rho = rho_of_z(xyz[:, 2])
    kappa0, _, _ = kappa0_and_density(box)
    return Atmosphere(xyz=xyz, T=np.ascontiguousarray(T), rho=np.ascontiguousarray(rho),
                      kappa0=float(kappa0), box=box, seed=seed)
