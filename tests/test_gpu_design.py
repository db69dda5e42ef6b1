"""The searchlight beam test (Sect. 3.1) on the GPU: with chi = S = 0 the
formal solution only carries the bottom boundary along the Delaunay lines
(or the regular grid's interpolated short characteristics). The GPU matches
the FP64 oracle to 1e-12 on both grids, and the beam arrives displaced by
tan(theta) times the box height (its centre within a cell and a half). The
beam is a 0/1 pattern, so the bar is on the error relative to the beam
intensity: rounding-level interpolation weights (1e-16) may leave 1e-15 on
one side and an exact zero on the other."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, to_dev
from synth import design

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    import paper_2306_01041_amd

    return paper_2306_01041_amd.load()


@pytest.fixture(scope="module")
def ctx(v):
    c = v.Context(0)
    yield c
    c.close()


def _err(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _centre(I, x):
    return (np.angle(np.sum(I * np.exp(2j * np.pi * x))) / (2 * np.pi)) % 1.0


@pytest.mark.parametrize("theta", [20.0, 45.0])
def test_searchlight_matches_oracle_and_geometry(v, ctx, theta):
    flush(f"searchlight {theta} deg")
    n_side = 21
    xyz, lo, hi, _, _, beam = design.searchlight(n_side=n_side, seed=7, radius=0.25)
    th = np.deg2rad(theta)
    d, w = np.array([[np.sin(th), 0.0, np.cos(th)]]), np.array([1.0])
    want = (0.5 + np.tan(th)) % 1.0
    f64 = torch.float64
    # Voronoi grid of uniformly random sites
    g = synth.voronoi_neighbours(xyz, lo, hi, periodic_xy=True)
    Ib = beam(g.xyz[:, 0], g.xyz[:, 1])[:, None]
    zero = np.zeros((g.n, 1))
    _, Io = oracle.fs_voronoi(g, d, w, oracle.select(g, d), zero, zero, Ib, keep_I=True)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(d, w)
    J = torch.empty((g.n, 1), dtype=f64, device="cuda:0")
    I = torch.empty((1, g.n, 1), dtype=f64, device="cuda:0")
    v.formal_solution(G, to_dev(zero, f64), to_dev(zero, f64), J, I_bottom=to_dev(Ib, f64), I_rays=I)
    torch.cuda.synchronize()
    Ig = I.cpu().numpy()
    assert _err(Ig, Io) <= 1e-12
    _, top = G.emergent_index()
    c = _centre(Ig[0, top, 0], g.xyz[top, 0])
    flush(f"  Voronoi: peak {Ig[0, top, 0].max():.3f}, centre {c:.3f} (want {want:.3f})")
    assert abs((c - want + 0.5) % 1.0 - 0.5) < 1.5 / n_side
    G.close()
    # regular lattice
    m = n_side ** 3
    dx = 1.0 / n_side
    z = np.linspace(0.0, 1.0, n_side)
    X, Y = np.meshgrid(np.arange(n_side) * dx, np.arange(n_side) * dx, indexing="xy")
    Ibr = np.zeros((m, 1))
    Ibr[: n_side * n_side, 0] = beam(X.ravel(), Y.ravel())
    zr = np.zeros((m, 1))
    _, Ior = oracle.fs_regular(n_side, n_side, z, dx, dx, d, w, zr, zr, Ibr, keep_I=True)
    Gr = v.Grid.regular(ctx, n_side, n_side, z, dx, dx)
    Gr.set_rays(d, w)
    J = torch.empty((m, 1), dtype=f64, device="cuda:0")
    I = torch.empty((1, m, 1), dtype=f64, device="cuda:0")
    v.formal_solution(Gr, to_dev(zr, f64), to_dev(zr, f64), J, I_bottom=to_dev(Ibr, f64), I_rays=I)
    torch.cuda.synchronize()
    Ir = I.cpu().numpy()
    assert _err(Ir, Ior) <= 1e-12
    topr = Ir[0, (n_side - 1) * n_side * n_side:, 0]
    c = _centre(topr, X.ravel())
    flush(f"  regular: peak {topr.max():.3f}, centre {c:.3f}")
    assert abs((c - want + 0.5) % 1.0 - 0.5) < 1.5 / n_side
    Gr.close()
