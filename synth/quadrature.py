"""Fixed angle quadratures (inputs to the solver).

The paper integrates the intensity over a fixed quadrature rather than random
directions (Sect. 2.5). Its node table (12 rays, L = 7, from a cited external
paper) is not reproduced here; the stand-in is a product rule: Gauss-Legendre
nodes in mu on (0, 1], equally spaced azimuths offset by half a step so that no
ray lies along the x or y axis, and both hemispheres.
"""

from __future__ import annotations

import numpy as np


def gauss_legendre_quadrature(n_mu: int = 3, n_phi: int = 4):
    """Return ``(dirs [R,3] float64, weights [R] float64)`` with R = 2*n_mu*n_phi.

    Ray order: upward hemisphere first (mu > 0), then downward; within a
    hemisphere mu ascending, then azimuth ascending. Each ray's weight is
    w_mu / (2 * n_phi) so the weights sum to one (J is the plain angle mean).
    """
    x, w = np.polynomial.legendre.leggauss(n_mu)
    mus = 0.5 * (x + 1.0)  # map [-1, 1] -> [0, 1]
    wmu = 0.5 * w          # sums to 1 on [0, 1]
    dirs = []
    wts = []
    for hemi in (+1.0, -1.0):
        for m, wm in zip(mus, wmu):
            st = np.sqrt(1.0 - m * m)
            for j in range(n_phi):
                phi = (j + 0.5) * 2.0 * np.pi / n_phi
                dirs.append((st * np.cos(phi), st * np.sin(phi), hemi * m))
                wts.append(wm / (2.0 * n_phi))
    return np.asarray(dirs, dtype=np.float64), np.asarray(wts, dtype=np.float64)


def vertical_quadrature():
    """Two rays, straight up and straight down, weight 1/2 each."""
    dirs = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], dtype=np.float64)
    return dirs, np.array([0.5, 0.5], dtype=np.float64)
