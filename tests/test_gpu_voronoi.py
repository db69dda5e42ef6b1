"""GPU parity of the Voronoi-grid path against the FP64 oracle.

Integer outputs (upwind sites, levels, sweep order) must be bit-identical;
FP64 intensities and J agree to 1e-12 relative; the FP32 sweep agrees with
the FP64 oracle to 1e-5 relative on J (its inputs are the FP64 fields rounded
to single precision). Every case runs through the C ABI.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, recipe_grid, relerr, to_dev, wavelengths

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    import paper_2306_01041_amd

    return paper_2306_01041_amd.load()


@pytest.fixture(scope="module")
def ctx(v):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = v.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def quad():
    return synth.gauss_legendre_quadrature()


@pytest.fixture(scope="module")
def grids():
    return {n: recipe_grid(n, seed=1041 + n) for n in (1000, 16384)}


def _gpu_grid(v, ctx, g, dirs, w):
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w, 7.0)
    return G


@pytest.mark.parametrize("n", [1000, 16384])
def test_selection_and_schedule_bit_exact(v, ctx, quad, grids, n):
    flush(f"selection n={n}")
    atm, g = grids[n]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    sel = oracle.select(g, dirs)
    lev, order, ptrs, nlev = oracle.levels(g, dirs, sel)
    info = G.info()
    assert info["n_fallback"] == int(sel.n_fallback.sum())
    assert info["max_levels"] == int(nlev.max())
    for r in range(len(dirs)):
        s = G.schedule(r)
        assert np.array_equal(s["k1"], sel.k1[r]), r
        assert np.array_equal(s["k2"], sel.k2[r]), r
        assert relerr(s["w1"], sel.w1[r]) <= 1e-13
        assert relerr(s["ds1"], sel.ds1[r]) <= 1e-15
        assert relerr(s["ds2"], sel.ds2[r]) <= 1e-15
        assert np.array_equal(s["level"], lev[r])
        assert np.array_equal(s["order"], order[r])
        assert np.array_equal(s["level_ptr"], ptrs[r])
    G.close()


def _fields(atm, nl, seed):
    """Grey LTE-like opacity with a per-wavelength random modulation, so the
    wavelength lanes are not all equal."""
    lam = wavelengths(nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    rng = np.random.default_rng(seed)
    chi = chi * rng.uniform(0.5, 2.0, size=(1, nl))
    return chi, S


@pytest.mark.parametrize("nl", [1, 3, 37, 101])
@pytest.mark.parametrize("mode", ["PLAIN", "BATCHED", "GRAPH", "PERSISTENT"])
def test_fp64_formal_solution_matches_oracle(v, ctx, quad, grids, nl, mode):
    flush(f"fp64 fs nl={nl} mode={mode}")
    atm, g = grids[1000]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    sel = oracle.select(g, dirs)
    chi, S = _fields(atm, nl, nl)
    Ib = S * 1.1
    It = S * 0.01
    Jo, Io = oracle.fs_voronoi(g, dirs, w, sel, chi, S, Ib, I_top=It, keep_I=True)
    d = torch.float64
    J = torch.empty((g.n, nl), dtype=d, device="cuda:0")
    I = torch.empty((len(dirs), g.n, nl), dtype=d, device="cuda:0")
    args = (to_dev(chi, d), to_dev(S, d), J)
    ib, it = to_dev(Ib, d), to_dev(It, d)
    ex = getattr(v, "VRT_EXEC_" + mode)
    for rep in range(2 if mode in ("GRAPH", "PERSISTENT") else 1):
        v.formal_solution(G, *args, I_bottom=ib, I_top=it, I_rays=I, exec_mode=ex)
        G.device_status()
        assert relerr(I.cpu().numpy(), Io) <= 1e-12
        assert relerr(J.cpu().numpy(), Jo) <= 1e-12
    G.close()


def test_c0_lte_continuum_fp64(v, ctx, quad, grids):
    flush("c0 lte fp64")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    lam = np.array([500e-9])
    d = torch.float64
    T = to_dev(atm.T, d)
    rho = to_dev(atm.rho, d)
    chi = torch.empty((g.n, 1), dtype=d, device="cuda:0")
    S = torch.empty_like(chi)
    v.lte_continuum(G, lam, atm.kappa0, T, rho, chi, S)
    chi_o, S_o = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    torch.cuda.synchronize()
    assert relerr(chi.cpu().numpy(), chi_o) <= 1e-14
    assert relerr(S.cpu().numpy(), S_o) <= 1e-14
    sel = oracle.select(g, dirs)
    Jo, Io = oracle.fs_voronoi(g, dirs, w, sel, chi_o, S_o, S_o, keep_I=True)
    J = torch.empty_like(chi)
    I = torch.empty((len(dirs), g.n, 1), dtype=d, device="cuda:0")
    v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    assert relerr(J.cpu().numpy(), Jo) <= 1e-12
    assert relerr(I.cpu().numpy(), Io) <= 1e-12
    off, sites = G.emergent_index()
    want_sites = oracle.emergent_sites(g, dirs)
    for r in range(len(dirs)):
        assert np.array_equal(sites[off[r]:off[r + 1]], want_sites[r])
    em = torch.empty((int(off[-1]), 1), dtype=d, device="cuda:0")
    v.emergent_gather(G, em, I_rays=None)  # from the library's record of the last solution
    torch.cuda.synchronize()
    emh = em.cpu().numpy()
    for r in range(len(dirs)):
        assert relerr(emh[off[r]:off[r + 1]], Io[r, want_sites[r]]) <= 1e-12
    G.close()


@pytest.mark.parametrize("nl", [1, 3, 4, 8, 17, 37, 64, 101, 104])
def test_lte_and_emergent_gather_every_lane_width(v, ctx, quad, grids, nl):
    """The LTE source kernel gives each site a group of 1 to 64 lanes with 1 or
    16 bytes of wavelengths per lane, depending on the wavelength count: the opacity and
    the Planck source against the FP64 oracle in both precisions, and the
    gathered rows equal to the intensities they copy, read from the caller's
    rows and from the library's own (padded) rows."""
    flush(f"lte + emergent gather nl={nl}")
    atm, g = grids[1000]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    lam = wavelengths(nl)
    chi_o, S_o = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    T, rho = to_dev(atm.T, torch.float64), to_dev(atm.rho, torch.float64)
    for d, tol in ((torch.float64, 1e-14), (torch.float32, 1e-7)):
        chi = torch.empty((g.n, nl), dtype=d, device="cuda:0")
        S = torch.empty_like(chi)
        v.lte_continuum(G, lam, atm.kappa0, T, rho, chi, S)
        torch.cuda.synchronize()
        assert relerr(chi.cpu().numpy(), chi_o) <= tol
        assert relerr(S.cpu().numpy(), S_o) <= tol
    f = torch.float32
    J = torch.empty_like(chi)
    I = torch.empty((len(dirs), g.n, nl), dtype=f, device="cuda:0")
    off, sites = G.emergent_index()
    v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_GRAPH)
    em_lib = torch.empty((int(off[-1]), nl), dtype=f, device="cuda:0")
    v.emergent_gather(G, em_lib)
    v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_GRAPH)
    em = torch.empty_like(em_lib)
    v.emergent_gather(G, em, I_rays=I)
    torch.cuda.synchronize()
    Ih, emh = I.cpu().numpy(), em.cpu().numpy()
    for r in range(len(dirs)):
        assert np.array_equal(emh[off[r]:off[r + 1]], Ih[r, sites[off[r]:off[r + 1]]])
    assert torch.equal(em, em_lib)
    # outputs that start 4 bytes past a 16-byte boundary take the one-element-per-lane
    # forms of both kernels and must give the same bits
    chi_m = torch.empty(g.n * nl + 1, dtype=f, device="cuda:0")[1:].view(g.n, nl)
    S_m = torch.empty(g.n * nl + 1, dtype=f, device="cuda:0")[1:].view(g.n, nl)
    v.lte_continuum(G, lam, atm.kappa0, T, rho, chi_m, S_m)
    em_m = torch.empty(int(off[-1]) * nl + 1, dtype=f, device="cuda:0")[1:].view(int(off[-1]), nl)
    v.emergent_gather(G, em_m, I_rays=I)
    torch.cuda.synchronize()
    assert torch.equal(chi_m, chi) and torch.equal(S_m, S)
    assert torch.equal(em_m, em)
    G.close()


@pytest.mark.parametrize("nl", [1, 64])
def test_fp32_batched_matches_fp64_oracle(v, ctx, quad, grids, nl):
    flush(f"fp32 vs oracle nl={nl}")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    lam = wavelengths(nl)
    chi_o, S_o = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    sel = oracle.select(g, dirs)
    Jo, Io = oracle.fs_voronoi(g, dirs, w, sel, chi_o, S_o, S_o, keep_I=True)
    f = torch.float32
    chi = torch.empty((g.n, nl), dtype=f, device="cuda:0")
    S = torch.empty_like(chi)
    v.lte_continuum(G, lam, atm.kappa0, to_dev(atm.T, torch.float64), to_dev(atm.rho, torch.float64), chi, S)
    J = torch.empty_like(chi)
    I = torch.empty((len(dirs), g.n, nl), dtype=f, device="cuda:0")
    v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    eJ = relerr(J.cpu().numpy(), Jo)
    eI = relerr(I.cpu().numpy(), Io)
    flush(f"  fp32 max rel err J {eJ:.3e} I {eI:.3e}")
    assert eJ <= 1e-5
    assert eI <= 1e-4
    G.close()


@pytest.mark.parametrize("chains", [1, 3])
def test_graph_replays_match_eager(v, ctx, quad, grids, chains):
    """A captured launch sequence (with forked streams when the rays are split
    into chains) replayed several times, with eager work and synchronisations
    between replays, reproduces the eager result bit for bit."""
    flush(f"graph replay chains={chains}")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    G.tune(v.VRT_TUNE_CHAINS, chains)
    chi_o, S_o = _fields(atm, 8, 3)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    J0 = torch.empty_like(chi)
    v.formal_solution(G, chi, S, J0, exec_mode=v.VRT_EXEC_BATCHED)
    torch.cuda.synchronize()
    ref = J0.cpu().numpy().copy()
    J = torch.empty_like(chi)
    for rep in range(4):
        J.fill_(-1.0)
        v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_GRAPH)
        torch.cuda.synchronize()
        assert np.array_equal(J.cpu().numpy(), ref), rep
        # eager work in between
        v.formal_solution(G, chi, S, J0, exec_mode=v.VRT_EXEC_PLAIN)
        torch.cuda.synchronize()
        assert np.array_equal(J0.cpu().numpy(), ref)
    G.close()


def test_tiny_lattice_and_fallback_grids(v, ctx, quad):
    flush("tiny lattice")
    dirs, w = quad
    g = synth.lattice_grid(2, 2, [0.0, 0.4, 1.0])
    G = _gpu_grid(v, ctx, g, dirs, w)
    sel = oracle.select(g, dirs)
    rng = np.random.default_rng(0)
    chi = rng.uniform(0.1, 2.0, (g.n, 2))
    S = rng.uniform(0.5, 3.0, (g.n, 2))
    Jo = oracle.fs_voronoi(g, dirs, w, sel, chi, S, S)
    d = torch.float64
    J = torch.empty((g.n, 2), dtype=d, device="cuda:0")
    v.formal_solution(G, to_dev(chi, d), to_dev(S, d), J, exec_mode=v.VRT_EXEC_BATCHED)
    torch.cuda.synchronize()
    assert relerr(J.cpu().numpy(), Jo) <= 1e-13
    for r in range(len(dirs)):
        s = G.schedule(r)
        assert np.array_equal(s["k1"], sel.k1[r])
    G.close()


@pytest.mark.parametrize("shape", [(1, 1, (0.0, 1.0)), (3, 2, (0.5,)), (1, 2, (0.0, 0.5, 1.0)),
                                   (2, 3, (0.0, 0.3, 1.0))])
def test_degenerate_grids_and_quadratures(v, ctx, quad, shape):
    """Degenerate cases of the method: two sites that are their own periodic
    neighbours, a single layer (every site on both walls: up rays return
    I_bottom, down rays 0), one-site-wide columns; with the full quadrature, a
    single oblique ray and one ray pair; every launch mode and layout, in FP64
    against the oracle and in FP32 within its tolerance. A wavelength count of
    zero is an argument error."""
    nx, ny, z = shape
    flush(f"degenerate grid {nx}x{ny}x{len(z)}")
    g = synth.lattice_grid(nx, ny, list(z))
    th = np.radians(40.0)
    oblique = np.array([[np.sin(th) * np.cos(0.3), np.sin(th) * np.sin(0.3), np.cos(th)]])
    pair = np.array([[0.0, np.sin(th), np.cos(th)], [0.0, -np.sin(th), -np.cos(th)]])
    rng = np.random.default_rng(len(z) + 7 * nx)
    nl = 3
    chi = rng.uniform(0.2, 3.0, (g.n, nl))
    S = rng.uniform(0.5, 2.0, (g.n, nl))
    for dirs, w in (quad, (oblique, np.array([1.0])), (pair, np.array([0.5, 0.5]))):
        sel = oracle.select(g, dirs)
        Jo = oracle.fs_voronoi(g, dirs, w, sel, chi, S, S)
        for shared, il in ((0, 0), (1, 0), (1, 1), (1, 2)):
            G = v.Grid.from_synth(ctx, g)
            G.tune(v.VRT_TUNE_SHARED_LEVELS, shared)
            G.set_rays(dirs, w, 7.0)
            G.tune(v.VRT_TUNE_INTERLEAVE, il)
            for d, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
                c_d, s_d = to_dev(chi, d), to_dev(S, d)
                for mode in (v.VRT_EXEC_PLAIN, v.VRT_EXEC_GRAPH, v.VRT_EXEC_PERSISTENT):
                    for rows in (False, True):
                        J = torch.full((g.n, nl), -1.0, dtype=d, device="cuda:0")
                        I = torch.empty((len(dirs), g.n, nl), dtype=d, device="cuda:0") if rows else None
                        v.formal_solution(G, c_d, s_d, J, I_rays=I, exec_mode=mode)
                        G.device_status()
                        e = relerr(J.cpu().numpy(), Jo)
                        assert e <= tol, (shape, len(dirs), shared, il, d, mode, rows, e)
            with pytest.raises(v.VrtError) as err:
                e0 = torch.empty((g.n, 0), dtype=torch.float64, device="cuda:0")
                v.formal_solution(G, e0, e0, torch.empty_like(e0))
            assert err.value.status == v.VRT_E_ARG
            G.close()


def test_determinism(v, ctx, quad, grids):
    flush("determinism")
    atm, g = grids[1000]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, 64, 9)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    out = []
    for mode in (v.VRT_EXEC_PLAIN, v.VRT_EXEC_BATCHED, v.VRT_EXEC_GRAPH, v.VRT_EXEC_BATCHED):
        J = torch.empty_like(chi)
        v.formal_solution(G, chi, S, J, exec_mode=mode)
        torch.cuda.synchronize()
        out.append(J.cpu().numpy())
    for o in out[1:]:
        assert np.array_equal(o, out[0])
    G.close()


def test_errors_do_not_launch(v, ctx, quad, grids):
    atm, g = grids[1000]
    G = v.Grid.from_synth(ctx, g)
    chi = torch.zeros((g.n, 1), dtype=torch.float64, device="cuda:0")
    with pytest.raises(v.VrtError) as e:
        v.formal_solution(G, chi, chi, chi)
    assert e.value.status == v.VRT_E_STATE
    dirs, w = quad
    with pytest.raises(v.VrtError) as e:
        G.set_rays(dirs, w * 2.0)
    assert e.value.status == v.VRT_E_ARG
    bad = dirs.copy()
    bad[0] = [1.0, 0.0, 0.0]
    with pytest.raises(v.VrtError):
        G.set_rays(bad, w)
    G.close()


def test_tuning_knobs_do_not_change_results(v, ctx, quad, grids):
    """Record order, die-chunk mapping, interleaved record copies and the
    pipelined kernel only reorder independent work: the results are
    bit-identical for every setting, and the autotuner reports every candidate
    (level-step layouts and the persistent sweep) and keeps the fastest."""
    flush("tuning knobs")
    atm, g = grids[16384]
    dirs, w = quad
    chi_o, S_o = _fields(atm, 64, 5)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    ref = None
    for order in (0, 1):
        for xcd, aff, ch, lb, rg, il, pp in ((0, 0, 1, 16, 1, 0, 0), (3, 0, 1, 16, 1, 0, 0), (8, 0, 1, 16, 1, 0, 0),
                                             (8, 1, 1, 16, 1, 0, 0), (8, 0, 2, 16, 1, 0, 0), (0, 0, 3, 16, 1, 0, 0),
                                             (8, 0, 5, 16, 1, 0, 0), (8, 0, 1, 32, 1, 0, 0), (8, 1, 1, 32, 1, 0, 0),
                                             (8, 0, 1, 16, 3, 0, 0), (8, 0, 1, 16, 5, 0, 0), (8, 0, 1, 16, 1, 1, 0),
                                             (0, 0, 1, 32, 1, 1, 0), (8, 0, 2, 16, 1, 1, 0), (8, 0, 1, 16, 1, 2, 0),
                                             (0, 0, 1, 16, 1, 2, 2), (8, 0, 1, 16, 1, 0, 2), (8, 0, 1, 16, 1, 1, 4),
                                             (8, 0, 3, 16, 1, 0, 8), (8, 0, 1, 16, 3, 0, 2)):
            G = v.Grid.from_synth(ctx, g)
            G.tune(v.VRT_TUNE_RECORD_ORDER, order)
            G.tune(v.VRT_TUNE_XCD_CHUNKS, xcd)
            G.tune(v.VRT_TUNE_RAY_AFFINITY, aff)
            G.tune(v.VRT_TUNE_CHAINS, ch)
            G.tune(v.VRT_TUNE_LANE_BYTES, lb)
            G.tune(v.VRT_TUNE_RAY_GROUPS, rg)
            G.tune(v.VRT_TUNE_INTERLEAVE, il)  # before the rays: built with the schedule
            G.tune(v.VRT_TUNE_PIPELINE, pp)
            G.set_rays(dirs, w)
            J = torch.empty_like(chi)
            for mode in (v.VRT_EXEC_GRAPH, v.VRT_EXEC_BATCHED, v.VRT_EXEC_PLAIN):
                v.formal_solution(G, chi, S, J, exec_mode=mode)
                torch.cuda.synchronize()
                out = J.cpu().numpy()
                if ref is None:
                    ref = out
                assert np.array_equal(out, ref), (order, xcd, aff, ch, lb, rg, il, pp, mode)
            G.close()
    for il, pp, ch in ((0, 0, 1), (1, 2, 1), (2, 2, 1), (2, 0, 1), (0, 0, 3)):
        G = v.Grid.from_synth(ctx, g)
        G.tune(v.VRT_TUNE_SHARED_LEVELS, 1)
        G.tune(v.VRT_TUNE_CHAINS, ch)
        G.set_rays(dirs, w)
        G.tune(v.VRT_TUNE_INTERLEAVE, il)
        G.tune(v.VRT_TUNE_PIPELINE, pp)
        J = torch.empty_like(chi)
        for mode in (v.VRT_EXEC_GRAPH, v.VRT_EXEC_BATCHED, v.VRT_EXEC_PLAIN, v.VRT_EXEC_PERSISTENT):
            v.formal_solution(G, chi, S, J, exec_mode=mode)
            G.device_status()
            assert np.array_equal(J.cpu().numpy(), ref), ("shared", il, pp, ch, mode)
        # the persistent sweep into caller rows (epoch stamps; with an interleaved
        # copy its wave items mix rays)
        I = torch.empty((len(dirs), g.n, chi.shape[1]), dtype=chi.dtype, device="cuda:0")
        v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_PERSISTENT)
        G.device_status()
        assert np.array_equal(J.cpu().numpy(), ref), ("shared, caller rows", il, pp, ch)
        G.close()
    # switched on after the rays are set: the copy is built at once
    G = _gpu_grid(v, ctx, g, dirs, w)
    G.tune(v.VRT_TUNE_INTERLEAVE, 1)
    J = torch.empty_like(chi)
    v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    assert np.array_equal(J.cpu().numpy(), ref)
    G.close()
    G = _gpu_grid(v, ctx, g, dirs, w)
    J = torch.empty_like(chi)
    rep = v.autotune(G, chi, S, J, reps=2)
    # per record order: 7 level-step layouts without the interleaved copies and
    # the persistent sweep, plus 5 with them under the Morton order; then 5
    # layouts with levels shared by the rays of one azimuth
    assert len(rep["candidates"]) == 28
    assert sum(c["shared_levels"] for c in rep["candidates"]) == 7
    assert {c["exec"] for c in rep["candidates"]} == {"graph", "persistent"}
    assert rep["chosen"]["ms"] == min(c["ms"] for c in rep["candidates"] if c["ms"] is not None)
    for mode in (v.VRT_EXEC_AUTO, v.VRT_EXEC_GRAPH, v.VRT_EXEC_PERSISTENT):
        v.formal_solution(G, chi, S, J, exec_mode=mode)
        G.device_status()
        assert np.array_equal(J.cpu().numpy(), ref), mode
    with pytest.raises(v.VrtError):
        G.tune(99, 1)
    G.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nl", [3, 8])
def test_persistent_items_across_rays_bitwise(v, ctx, quad, grids, prec, nl):
    """Wave items cut from an interleaved record copy hold records of several
    rays (each lane addresses its own ray's rows): in both precisions, with
    whole 16-byte vectors (8 wavelengths) and single elements (3), into the
    library's sign-encoded rows and into caller rows with epoch stamps, the
    persistent sweep gives the level steps' J and intensities bit for bit."""
    flush(f"persistent mixed items {prec} nl={nl}")
    atm, g = grids[16384]
    dirs, w = quad
    dt = torch.float32 if prec == "f32" else torch.float64
    chi_o, S_o = _fields(atm, nl, 21)
    chi, S = to_dev(chi_o, dt), to_dev(S_o, dt)
    R = len(dirs)
    G = v.Grid.from_synth(ctx, g)
    G.tune(v.VRT_TUNE_SHARED_LEVELS, 1)
    G.set_rays(dirs, w, 7.0)
    Jg = torch.empty_like(chi)
    Ig = torch.empty((R, g.n, nl), dtype=dt, device="cuda:0")
    v.formal_solution(G, chi, S, Jg, I_rays=Ig, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    for il in (1, 2):
        G.tune(v.VRT_TUNE_INTERLEAVE, il)
        for _ in range(2):
            J = torch.full_like(chi, -1.0)
            v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
            G.device_status()
            assert torch.equal(J, Jg), ("own rows", il)
            I = torch.full_like(Ig, -1.0)
            v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_PERSISTENT)
            G.device_status()
            assert torch.equal(J, Jg) and torch.equal(I, Ig), ("caller rows", il)
    G.close()


@pytest.mark.parametrize("nl", [1, 64, 101])
def test_persistent_fp32_matches_graph_bitwise(v, ctx, quad, grids, nl):
    """The persistent dataflow sweep performs the same arithmetic per record as
    the level-synchronous launches, so its results are bit-identical."""
    flush(f"persistent fp32 nl={nl}")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, nl, 11)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    Jg = torch.empty_like(chi)
    v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    ref = Jg.cpu().numpy()
    for rep in range(3):
        J = torch.full_like(chi, -1.0)
        v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
        G.device_status()
        assert np.array_equal(J.cpu().numpy(), ref), rep
    G.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_shared_levels_give_identical_results(v, ctx, quad, grids, prec):
    """One level schedule shared by the rays of one hemisphere and azimuth is a
    valid schedule for each of them (a site's level is the same for the group
    and above the level of every site any of them reads from), is at least as
    deep as each ray's own, and gives the per-ray schedule's intensities, J and
    adjoint bit for bit in every launch mode."""
    flush(f"shared levels {prec}")
    atm, g = grids[16384]
    dirs, w = quad
    dt = torch.float32 if prec == "f32" else torch.float64
    chi_o, S_o = _fields(atm, 8, 13)
    chi, S = to_dev(chi_o, dt), to_dev(S_o, dt)
    R = len(dirs)
    out = {}
    own = {}
    for shared in (0, 1):
        G = v.Grid.from_synth(ctx, g)
        G.tune(v.VRT_TUNE_SHARED_LEVELS, shared)
        G.set_rays(dirs, w, 7.0)
        sch = [G.schedule(r) for r in range(R)]
        if shared:
            hz = np.hypot(dirs[:, 0], dirs[:, 1])
            for r in range(R):
                k1, k2, lev = sch[r]["k1"], sch[r]["k2"], sch[r]["level"]
                for k in (k1, k2):
                    m = k >= 0
                    assert np.all(lev[m] > lev[k[m]]), r
                assert np.all(lev[k1 < 0] == 0), r
                assert sch[r]["n_levels"] >= own[r], r
                for q in range(R):
                    if np.sign(dirs[q, 2]) == np.sign(dirs[r, 2]) and np.allclose(dirs[q, :2] / hz[q], dirs[r, :2] / hz[r]):
                        assert np.array_equal(sch[q]["level"], lev), (r, q)
        else:
            own = {r: sch[r]["n_levels"] for r in range(R)}
        res = []
        for mode in (v.VRT_EXEC_PLAIN, v.VRT_EXEC_GRAPH, v.VRT_EXEC_PERSISTENT):
            J = torch.empty_like(chi)
            I = torch.empty((R, g.n, 8), dtype=dt, device="cuda:0")
            v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=mode)
            G.device_status()
            res += [J.cpu().numpy(), I.cpu().numpy()]
        gI = torch.ones((R, g.n, 8), dtype=dt, device="cuda:0")
        res += [t.cpu().numpy() for t in v.formal_solution_vjp(G, chi, S, dL_dI=gI, I_rays=I)]
        out[shared] = res
        G.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nl", [64, 101])
@pytest.mark.parametrize("blocks", [8, 8192])
def test_persistent_any_grid_size_gives_the_same_result(v, ctx, quad, grids, nl, blocks):
    """Work goes only to wavefronts that registered before the count was
    frozen, so a grid of 8 workgroups, and one of 8192 (several times what can
    be resident: the late workgroups take no work), give the graph sweep's
    intensities bit for bit."""
    flush(f"persistent grid of {blocks} workgroups nl={nl}")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, nl, 13)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    Jg = torch.empty_like(chi)
    v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    G.tune(v.VRT_TUNE_PERSIST_BLOCKS, blocks)
    for rep in range(2):
        J = torch.full_like(chi, -1.0)
        v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
        G.device_status()
        assert np.array_equal(J.cpu().numpy(), Jg.cpu().numpy()), rep
    G.close()


def test_persistent_sign_encoded_rows_across_modes_and_layouts(v, ctx, quad, grids):
    """Without caller rows the persistent sweep keeps its own sign-encoded rows
    (odd epochs store -I). Solutions of changing precision and wavelength count,
    interleaved with graph-launched and stamped (caller-row) persistent solutions,
    must each give the graph sweep's J and emergent rows bit for bit."""
    flush("persistent sign-encoded rows")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    off, _ = G.emergent_index()
    for d, nl in ((torch.float32, 64), (torch.float32, 5), (torch.float64, 3), (torch.float32, 64)):
        chi_o, S_o = _fields(atm, nl, 17 + nl)
        chi, S = to_dev(chi_o, d), to_dev(S_o, d)
        Jg = torch.empty_like(chi)
        v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
        em_g = torch.empty((int(off[-1]), nl), dtype=d, device="cuda:0")
        v.emergent_gather(G, em_g)
        I = torch.empty((len(dirs), g.n, nl), dtype=d, device="cuda:0")
        for rep in range(4):
            J = torch.full_like(chi, -1.0)
            if rep == 2:  # caller rows: the stamped protocol, plain positive rows
                v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=v.VRT_EXEC_PERSISTENT)
            else:
                v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
            em = torch.empty_like(em_g)
            v.emergent_gather(G, em, I_rays=I if rep == 2 else None)
            G.device_status()
            assert torch.equal(J, Jg), (d, nl, rep)
            assert torch.equal(em, em_g), (d, nl, rep)
            if rep == 2:
                assert bool((I >= 0).all())
    G.close()


def test_persistent_sign_encoding_rejects_negative_intensities(v, ctx, quad, grids):
    """A negative source function gives negative intensities, which the sign
    encoding cannot carry: the sweep still drains, the device status reports a
    numeric error once, and the next solution of valid inputs is correct."""
    flush("persistent sign-encoded rows, negative source")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, 8, 19)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    Jg = torch.empty_like(chi)
    v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
    Sneg = -S  # every boundary intensity (I_bottom defaults to S) is negative
    J = torch.empty_like(chi)
    v.formal_solution(G, chi, Sneg, J, exec_mode=v.VRT_EXEC_PERSISTENT)
    with pytest.raises(v.VrtError) as e:
        G.device_status()
    assert e.value.status == v.VRT_E_NUMERIC
    G.device_status()  # cleared
    for _ in range(2):
        v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
        G.device_status()
        assert torch.equal(J, Jg)
    G.close()


def test_persistent_error_state_is_never_stale(v, ctx, quad, grids):
    """An error left by a sign-encoded sweep must never let later results come
    from rows of an older epoch. After a sweep with negative intensities
    (unacknowledged), a second sign-encoded solution does not run: its J and
    emergent intensities come back as NaN rather than as the previous rows. A
    persistent two-level solve then reports the pending error with its own
    code (numeric, not a timeout) and acknowledges it, and the next valid
    sign-encoded solution equals the graph-launched one bit for bit."""
    from synth.nlte import LAMBDA0_NM, line_setup

    flush("persistent error state: sign-encoded, then two-level")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, 8, 23)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    Jg = torch.empty_like(chi)
    v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
    em_g = torch.empty((G.emergent_index()[0][-1], 8), dtype=f, device="cuda:0")
    v.emergent_gather(G, em_g)
    J = torch.empty_like(chi)
    v.formal_solution(G, chi, -S, J, exec_mode=v.VRT_EXEC_PERSISTENT)  # sets the numeric error
    assert bool(torch.isnan(J).all())
    v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)  # error still pending: does not run
    torch.cuda.synchronize()
    assert bool(torch.isnan(J).all())
    em = torch.empty_like(em_g)
    v.emergent_gather(G, em)
    torch.cuda.synchronize()
    assert bool(torch.isnan(em).all())
    # a persistent two-level solve reports the pending error as numeric
    line = line_setup(atm.T, atm.rho, n_lambda=9)
    d = torch.float64
    chi_c = torch.empty((g.n, 1), dtype=d, device="cuda:0")
    B = torch.empty_like(chi_c)
    v.lte_continuum(G, np.array([LAMBDA0_NM * 1e-9]), atm.kappa0, to_dev(atm.T, d), to_dev(atm.rho, d), chi_c, B)
    chi_c, B = chi_c[:, 0].contiguous(), B[:, 0].contiguous()
    S_L = B.clone()
    with pytest.raises(v.VrtError) as e:
        v.two_level_solve(G, line.wlam, to_dev(line.phi, d), to_dev(line.chi_line, d), chi_c, B, 1e-2, S_L,
                          max_iter=3, tol=1e-3, sweep_dtype=f, exec_mode=v.VRT_EXEC_PERSISTENT)
    assert e.value.status == v.VRT_E_NUMERIC
    G.device_status()  # acknowledged by the solve
    for _ in range(3):
        v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
        G.device_status()
        assert torch.equal(J, Jg)
        v.emergent_gather(G, em)
        assert torch.equal(em, em_g)
    G.close()


def test_persistent_bounded_wait_reports_timeout(v, ctx, quad, grids):
    """A spin bound of zero polls makes the first unmet wait give up: the kernel
    still drains, the device status reports a timeout once, and the next
    solution with the normal bound is correct again."""
    flush("persistent timeout path")
    atm, g = grids[16384]
    dirs, w = quad
    G = _gpu_grid(v, ctx, g, dirs, w)
    chi_o, S_o = _fields(atm, 8, 12)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    Jg = torch.empty_like(chi)
    v.formal_solution(G, chi, S, Jg, exec_mode=v.VRT_EXEC_GRAPH)
    torch.cuda.synchronize()
    G.tune(v.VRT_TUNE_SPIN_CAP, 0)
    J = torch.empty_like(chi)
    v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
    with pytest.raises(v.VrtError) as e:
        G.device_status()
    assert e.value.status == v.VRT_E_TIMEOUT
    G.device_status()  # cleared
    G.tune(v.VRT_TUNE_SPIN_CAP, 1 << 22)
    v.formal_solution(G, chi, S, J, exec_mode=v.VRT_EXEC_PERSISTENT)
    G.device_status()
    assert np.array_equal(J.cpu().numpy(), Jg.cpu().numpy())
    G.close()


@pytest.mark.parametrize("n_mu,n_phi", [(1, 3), (2, 5)])
def test_ray_affinity_and_chains_with_uneven_rays(v, ctx, grids, n_mu, n_phi):
    """6 and 20 rays leave dies with different numbers of rays (or none) and
    chains with different numbers of rays: the affinity tables and the chain
    ranges must still cover every record once; the intensities of every ray
    equal those of the plain block order bit for bit."""
    flush(f"ray affinity n_mu={n_mu} n_phi={n_phi}")
    atm, g = grids[16384]
    dirs, w = synth.gauss_legendre_quadrature(n_mu=n_mu, n_phi=n_phi)
    chi_o, S_o = _fields(atm, 8, 3)
    f = torch.float32
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    outs = []
    for aff, ch, mode in ((0, 1, "BATCHED"), (1, 1, "BATCHED"), (0, 4, "BATCHED"), (0, 1, "PERSISTENT")):
        G = v.Grid.from_synth(ctx, g)
        G.tune(v.VRT_TUNE_RAY_AFFINITY, aff)
        G.tune(v.VRT_TUNE_CHAINS, ch)
        G.set_rays(dirs, w)
        J = torch.empty_like(chi)
        I = torch.full((len(dirs), g.n, 8), float("nan"), dtype=f, device="cuda:0")
        v.formal_solution(G, chi, S, J, I_rays=I, exec_mode=getattr(v, "VRT_EXEC_" + mode))
        G.device_status()
        outs.append(I.cpu().numpy())
        G.close()
    for o in outs[1:]:
        assert np.all(np.isfinite(o))
        assert np.array_equal(outs[0], o)


def test_grid_outliving_its_context(v, quad, grids):
    """Destroying a context frees its grids; closing such a grid afterwards is
    a no-op (no use of the freed context)."""
    flush("grid outliving context")
    atm, g = grids[1000]
    dirs, w = quad
    c = v.Context(0)
    G = _gpu_grid(v, c, g, dirs, w)
    c.close()
    G.close()
    assert G.handle is None
