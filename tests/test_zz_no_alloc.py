"""The entry point that allocates nothing (vrt_formal_solution_noalloc),
through the C ABI: its J equals vrt_formal_solution's (batched mode, the same
kernels) bit for bit on two calls in a row, the second smaller, in both
precisions; sizes beyond its static buffer are rejected before any work."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, recipe_grid, to_dev, wavelengths

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    import paper_2306_01041_amd

    return paper_2306_01041_amd.load()


def _fields(atm, nl, seed):
    chi, S = oracle.lte(wavelengths(nl), atm.kappa0, atm.T, atm.rho)
    chi = chi * np.random.default_rng(seed).uniform(0.5, 2.0, (1, nl))
    return chi, S


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_formal_solution(v, prec):
    dt = torch.float32 if prec == "f32" else torch.float64
    ctx = v.Context(0)
    dirs, w = synth.gauss_legendre_quadrature()
    # two calls in a row: a larger grid and more wavelengths, then a smaller one
    for n, nl, seed in ((16384, 16, 5), (1000, 4, 6)):
        flush(f"no-alloc {prec}: {n} sites x {nl} wavelengths")
        atm, g = recipe_grid(n, seed=1041 + n)
        G = v.Grid.from_synth(ctx, g)
        G.set_rays(dirs, w)
        chi_o, S_o = _fields(atm, nl, seed)
        chi, S = to_dev(chi_o, dt), to_dev(S_o, dt)
        Jref = torch.empty_like(chi)
        v.formal_solution(G, chi, S, Jref, exec_mode=v.VRT_EXEC_BATCHED)
        J = torch.full_like(chi, float("nan"))
        v.formal_solution_noalloc(G, chi, S, J)
        torch.cuda.synchronize()
        assert torch.equal(J, Jref)
        G.close()
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_buffer(v):
    flush("no-alloc size limit")
    ctx = v.Context(0)
    dirs, w = synth.gauss_legendre_quadrature()
    atm, g = recipe_grid(16384, seed=1041 + 16384)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    nl = 64  # 24 rays x 16,384 sites x 64 wavelengths x 4 B = 96 MiB > 64 MiB
    chi = torch.ones((g.n, nl), dtype=torch.float32, device="cuda:0")
    J = torch.empty_like(chi)
    with pytest.raises(v.VrtError) as e:
        v.formal_solution_noalloc(G, chi, chi, J)
    assert e.value.status == v.VRT_E_ARG and "bytes" in str(e.value)
    G.close()
    ctx.close()
