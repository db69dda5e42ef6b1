"""Strided input rows (vrt_formal_solution_ld, vrt_lte_continuum_ld) on the GPU.

The strided entry points read the rows of site i of chi, S, I_bottom and
I_top at i * ld_src. The kernels' arithmetic does not depend on where a row
lives, so every result must equal that of the same values in separate
[n][n_lambda] arrays bit for bit: in every launch mode and record layout, for
the linear and the quadratic Bezier segment, in both precisions, with whole
16-byte vectors and with single elements per lane. The separate-array results
are themselves pinned to the oracle by the other parity tests.
"""

import numpy as np
import pytest

import oracle
from gpu_util import flush, recipe_grid, to_dev, wavelengths

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
def case():
    import synth

    atm, g = recipe_grid(4096, seed=77)
    dirs, w = synth.gauss_legendre_quadrature()
    return atm, g, dirs, w


def _fields(atm, nl, seed):
    lam = wavelengths(nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    rng = np.random.default_rng(seed)
    return chi * rng.uniform(0.5, 2.0, size=(1, nl)), S


def _rows(arrays, dt, pad=0):
    """The arrays as slots of one [n][k][nl + pad] device array: views whose
    rows lie k (nl + pad) elements apart."""
    n, nl = arrays[0].shape
    big = torch.full((n, len(arrays), nl + pad), float("nan"), dtype=dt, device="cuda:0")
    for k, a in enumerate(arrays):
        big[:, k, :nl] = to_dev(a, dt)
    return big, [big[:, k, :nl] for k in range(len(arrays))]


LAYOUTS = {
    # name: (knobs set before the rays, knobs set after)
    "default": ({}, {}),
    "shared levels, interleaved, pipelined": ({"SHARED_LEVELS": 1}, {"INTERLEAVE": 1, "PIPELINE": 2}),
    "site-order copy": ({}, {"INTERLEAVE": 2, "PIPELINE": 4}),
    "ray affinity": ({"RAY_AFFINITY": 1}, {}),
    "chains, 32-byte lanes": ({"CHAINS": 2, "LANE_BYTES": 32}, {}),
    "ray groups": ({"RAY_GROUPS": 3}, {}),
    "bezier": ({"SEGMENT": 1}, {}),
}


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nl", [3, 8, 13])
@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_strided_rows_equal_separate_arrays_bitwise(v, ctx, case, prec, nl, layout):
    flush(f"strided rows {prec} nl={nl} layout={layout}")
    atm, g, dirs, w = case
    dt = torch.float32 if prec == "f32" else torch.float64
    R = len(dirs)
    chi_o, S_o = _fields(atm, nl, nl)
    Ib_o, It_o = S_o * 1.1, S_o * 0.01
    sep = [to_dev(a, dt) for a in (chi_o, S_o, Ib_o, It_o)]
    before, after = LAYOUTS[layout]
    G = v.Grid.from_synth(ctx, g)
    for k, val in before.items():
        G.tune(getattr(v, "VRT_TUNE_" + k), val)
    G.set_rays(dirs, w, 7.0)
    for k, val in after.items():
        G.tune(getattr(v, "VRT_TUNE_" + k), val)
    # pairs (S also the bottom boundary: NULL I_bottom), and four rows per
    # site with padding (ld not a multiple of the vector width for nl = 13)
    _, pair = _rows([chi_o, S_o], dt)
    _, quad = _rows([chi_o, S_o, Ib_o, It_o], dt, pad=1)
    for mode in ("GRAPH", "BATCHED", "PLAIN", "PERSISTENT"):
        ex = getattr(v, "VRT_EXEC_" + mode)
        for inputs, bound in ((pair, False), (quad, True)):
            kw = {"I_bottom": inputs[2], "I_top": inputs[3]} if bound else {}
            kws = {"I_bottom": sep[2], "I_top": sep[3]} if bound else {}
            Jr = torch.full((g.n, nl), -1.0, dtype=dt, device="cuda:0")
            Ir = torch.full((R, g.n, nl), -1.0, dtype=dt, device="cuda:0")
            v.formal_solution(G, sep[0], sep[1], Jr, I_rays=Ir, exec_mode=ex, **kws)
            G.device_status()
            for rows in ("caller", "own"):
                for _ in range(2):  # the second call replays a captured graph
                    J = torch.full_like(Jr, -2.0)
                    I = torch.full_like(Ir, -2.0) if rows == "caller" else None
                    v.formal_solution(G, inputs[0], inputs[1], J, I_rays=I, exec_mode=ex, **kw)
                    G.device_status()
                    assert torch.equal(J, Jr), (mode, bound, rows)
                    if I is not None:
                        assert torch.equal(I, Ir), (mode, bound, rows)
            # the emergent intensities of the library's own rows
            em_s = torch.empty((int(G.emergent_index()[0][-1]), nl), dtype=dt, device="cuda:0")
            em_r = torch.empty_like(em_s)
            v.formal_solution(G, sep[0], sep[1], Jr, exec_mode=ex, **kws)
            v.emergent_gather(G, em_s)
            v.formal_solution(G, inputs[0], inputs[1], J, exec_mode=ex, **kw)
            v.emergent_gather(G, em_r)
            G.device_status()
            assert torch.equal(em_r, em_s), (mode, bound, "emergent")
    G.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nl", [3, 8, 64])
def test_lte_continuum_strided_rows(v, ctx, case, prec, nl):
    """The LTE assembly into paired rows writes the values it writes into
    separate arrays, bit for bit, and nothing between the rows."""
    flush(f"lte strided {prec} nl={nl}")
    atm, g, dirs, w = case
    dt = torch.float32 if prec == "f32" else torch.float64
    G = v.Grid.from_synth(ctx, g)
    lam = wavelengths(nl)
    T, rho = to_dev(atm.T, torch.float64), to_dev(atm.rho, torch.float64)
    chi = torch.empty((g.n, nl), dtype=dt, device="cuda:0")
    S = torch.empty_like(chi)
    v.lte_continuum(G, lam, atm.kappa0, T, rho, chi, S)
    big = torch.full((g.n, 2, nl + 3), 7.0, dtype=dt, device="cuda:0")
    v.lte_continuum(G, lam, atm.kappa0, T, rho, big[:, 0, :nl], big[:, 1, :nl])
    torch.cuda.synchronize()
    assert torch.equal(big[:, 0, :nl], chi) and torch.equal(big[:, 1, :nl], S)
    assert bool((big[:, :, nl:] == 7.0).all())
    G.close()


def test_strided_rows_errors(v, ctx, case):
    """Row strides below n_lambda, and strided rows on a regular grid, are
    argument errors that launch nothing; the grids still run afterwards."""
    import ctypes

    flush("strided rows errors")
    atm, g, dirs, w = case
    nl = 8
    f = torch.float32
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    chi_o, S_o = _fields(atm, nl, 3)
    chi, S = to_dev(chi_o, f), to_dev(S_o, f)
    J = torch.empty_like(chi)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = v.vrt_formal_solution_ld(G.handle, v.VRT_F32, v.VRT_EXEC_BATCHED, nl, nl - 1, p(chi), p(S), None, None, p(J),
                                  None)
    assert st == v.VRT_E_ARG
    lam = np.ascontiguousarray(wavelengths(nl))
    st = v.vrt_lte_continuum_ld(G.handle, v.VRT_F32, nl, nl - 1, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                1.0, p(to_dev(atm.T, torch.float64)), p(to_dev(atm.rho, torch.float64)), p(chi), p(S))
    assert st == v.VRT_E_ARG
    with pytest.raises(ValueError):
        v.formal_solution(G, chi, S.t().contiguous().t(), J)  # entries of a row not adjacent
    v.formal_solution(G, chi, S, J)
    torch.cuda.synchronize()
    G.close()
    nx, ny, nz = 4, 4, 5
    Rg = v.Grid.regular(ctx, nx, ny, np.linspace(0, 1, nz), 0.25, 0.25)
    Rg.set_rays(dirs, w)
    n = nx * ny * nz
    big = torch.ones((n, 2, nl), dtype=f, device="cuda:0")
    Jr = torch.empty((n, nl), dtype=f, device="cuda:0")
    with pytest.raises(v.VrtError) as e:
        v.formal_solution(Rg, big[:, 0], big[:, 1], Jr)
    assert e.value.status == v.VRT_E_ARG
    v.formal_solution(Rg, big[:, 0].contiguous(), big[:, 1].contiguous(), Jr)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Jr).all())
    Rg.close()
