"""GPU parity of the regular-grid short-characteristics solver (Sect. 2.6)
against the FP64 oracle, and of a lattice Voronoi grid against it for
vertical rays."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, relerr, to_dev

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


def _case(nx, ny, nz, nl, seed):
    rng = np.random.default_rng(seed)
    z = np.cumsum(np.r_[0.0, rng.uniform(0.05, 0.2, nz - 1)])
    n = nx * ny * nz
    chi = 10 ** rng.uniform(-1, 1.3, (n, nl))
    S = rng.uniform(0.5, 5.0, (n, nl))
    Ib = rng.uniform(0.5, 5.0, (n, nl))
    return z, chi, S, Ib


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["PLAIN", "GRAPH"])
@pytest.mark.parametrize("nl", [1, 5, 8, 70])
@pytest.mark.parametrize("shape", [(16, 12, 21), (13, 7, 9)])
def test_regular_matches_oracle(v, ctx, prec, mode, nl, shape):
    # (13, 7): rows that are not a multiple of the points a wavefront covers
    # (1 to 64 depending on the row length), so the last wavefront of each row
    # is partly idle
    flush(f"regular prec={prec} mode={mode} nl={nl} shape={shape}")
    nx, ny, nz = shape
    z, chi, S, Ib = _case(nx, ny, nz, nl, nl)
    dirs, w = synth.gauss_legendre_quadrature()
    Jo, Io = oracle.fs_regular(nx, ny, z, 0.11, 0.13, dirs, w, chi, S, Ib, keep_I=True)
    G = v.Grid.regular(ctx, nx, ny, z, 0.11, 0.13)
    G.set_rays(dirs, w)
    d = torch.float64 if prec == "f64" else torch.float32
    J = torch.empty((nx * ny * nz, nl), dtype=d, device="cuda:0")
    I = torch.empty((len(dirs), nx * ny * nz, nl), dtype=d, device="cuda:0")
    v.formal_solution(G, to_dev(chi, d), to_dev(S, d), J, I_bottom=to_dev(Ib, d), I_rays=I,
                      exec_mode=getattr(v, "VRT_EXEC_" + mode))
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "f64" else 1e-5
    eJ = relerr(J.cpu().numpy(), Jo)
    flush(f"  J err {eJ:.2e}")
    assert eJ <= tol
    assert relerr(I.cpu().numpy(), Io) <= (tol if prec == "f64" else 1e-4)
    off, sites = G.emergent_index()
    em = torch.empty((int(off[-1]), nl), dtype=d, device="cuda:0")
    v.emergent_gather(G, em, I_rays=I)
    torch.cuda.synchronize()
    emh = em.cpu().numpy()
    for r in range(len(dirs)):
        assert relerr(emh[off[r]:off[r + 1]], Io[r, sites[off[r]:off[r + 1]]]) <= (tol if prec == "f64" else 1e-4)
    G.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nl", [8, 24, 64])
def test_regular_modes_bitwise_equal(v, ctx, prec, nl):
    """One launch per ray and plane (plain) and one per plane for all rays
    (graph), with the LDS-tiled plane kernel and with the row kernel, run the
    same per-point arithmetic, so their intensities agree bit for bit (rows of
    13 and 9 points: partial 8 x 8 tiles; 24 wavelengths: a partial chunk)."""
    flush(f"regular plain vs graph, tiled vs rows {prec} nl={nl}")
    nx, ny, nz = 13, 9, 11
    z, chi, S, Ib = _case(nx, ny, nz, nl, 5)
    dirs, w = synth.gauss_legendre_quadrature()
    G = v.Grid.regular(ctx, nx, ny, z, 0.11, 0.13)
    G.set_rays(dirs, w)
    d = torch.float64 if prec == "f64" else torch.float32
    out = {}
    for tiled in (1, 0, 2):
        G.tune(v.VRT_TUNE_REGULAR_TILE, tiled)
        for mode in ("PLAIN", "GRAPH"):
            J = torch.empty((nx * ny * nz, nl), dtype=d, device="cuda:0")
            I = torch.empty((len(dirs), nx * ny * nz, nl), dtype=d, device="cuda:0")
            v.formal_solution(G, to_dev(chi, d), to_dev(S, d), J, I_bottom=to_dev(Ib, d), I_rays=I,
                              exec_mode=getattr(v, "VRT_EXEC_" + mode))
            out[(tiled, mode)] = (J, I)
    torch.cuda.synchronize()
    ref = out[(0, "PLAIN")]
    for key, (J, I) in out.items():
        assert torch.equal(I, ref[1]), key
        assert torch.equal(J, ref[0]), key
    G.close()


def test_lattice_voronoi_equals_regular_vertical_rays(v, ctx):
    flush("lattice vs regular")
    nx, ny, nz, nl = 8, 6, 15, 3
    z, chi, S, Ib = _case(nx, ny, nz, nl, 77)
    dirs, w = synth.vertical_quadrature()
    g = synth.lattice_grid(nx, ny, z, dx=0.3, dy=0.2)
    d = torch.float64
    Gv = v.Grid.from_synth(ctx, g)
    Gv.set_rays(dirs, w)
    Gr = v.Grid.regular(ctx, nx, ny, z, 0.3, 0.2)
    Gr.set_rays(dirs, w)
    Jv = torch.empty((g.n, nl), dtype=d, device="cuda:0")
    Jr = torch.empty_like(Jv)
    args = (to_dev(chi, d), to_dev(S, d))
    v.formal_solution(Gv, *args, Jv, I_bottom=to_dev(Ib, d))
    v.formal_solution(Gr, *args, Jr, I_bottom=to_dev(Ib, d))
    torch.cuda.synchronize()
    assert relerr(Jv.cpu().numpy(), Jr.cpu().numpy()) <= 1e-13
    Gv.close()
    Gr.close()


def test_regular_autotune_picks_a_plane_kernel(v, ctx):
    """On a regular grid the autotuner times the row and the LDS-tiled plane
    kernels, keeps the faster, and the results stay bit for bit the same."""
    flush("regular autotune")
    nx, ny, nz, nl = 24, 16, 20, 16
    z, chi, S, Ib = _case(nx, ny, nz, nl, 9)
    dirs, w = synth.gauss_legendre_quadrature()
    G = v.Grid.regular(ctx, nx, ny, z, 0.11, 0.13)
    G.set_rays(dirs, w)
    d = torch.float32
    c_d, S_d, Ib_d = to_dev(chi, d), to_dev(S, d), to_dev(Ib, d)
    J = torch.empty((nx * ny * nz, nl), dtype=d, device="cuda:0")
    v.formal_solution(G, c_d, S_d, J, I_bottom=Ib_d, exec_mode=v.VRT_EXEC_GRAPH)
    ref = J.clone()
    rep = v.autotune(G, c_d, S_d, J, I_bottom=Ib_d, reps=2)
    assert [c["regular_tile"] for c in rep["candidates"]] == [0, 1]
    assert rep["chosen"]["ms"] == min(c["ms"] for c in rep["candidates"])
    for mode in (v.VRT_EXEC_AUTO, v.VRT_EXEC_PLAIN):
        v.formal_solution(G, c_d, S_d, J, I_bottom=Ib_d, exec_mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(J, ref), mode
    G.close()
