"""GPU parity of the reverse sweep and the LTE chain rule against the oracle's
reverse sweep, and of the autograd gradient of an emergent-intensity misfit
against the oracle's gradient and against central differences."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, recipe_grid, relerr, to_dev

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


@pytest.fixture(scope="module")
def case():
    atm, g = recipe_grid(2000, seed=404)
    dirs, w = synth.gauss_legendre_quadrature()
    sel = oracle.select(g, dirs)
    return atm, g, dirs, w, sel


def normerr(a, b):
    """max |a - b| / max |b| (adjoint entries span many decades and cancel)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nl", [3, 64])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reverse_sweep_matches_oracle(v, ctx, case, nl, prec):
    flush(f"vjp nl={nl} prec={prec}")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    chi = chi * np.random.default_rng(nl).uniform(0.5, 2.0, (1, nl))
    rng = np.random.default_rng(1)
    gI = rng.standard_normal((len(dirs), g.n, nl))
    gJ = rng.standard_normal((g.n, nl))
    Jo, Io = oracle.fs_voronoi(g, dirs, w, sel, chi, S, S, keep_I=True)
    oc, oS, oIb, oIt = oracle.fs_voronoi_vjp(g, dirs, w, sel, chi, S, Io, dL_dI=gI, dL_dJ=gJ)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    dt = torch.float64 if prec == "f64" else torch.float32
    c_d, S_d = to_dev(chi, dt), to_dev(S, dt)
    J = torch.empty_like(c_d)
    I = torch.empty((len(dirs), g.n, nl), dtype=dt, device="cuda:0")
    v.formal_solution(G, c_d, S_d, J, I_rays=I)
    outs = v.formal_solution_vjp(G, c_d, S_d, dL_dI=to_dev(gI, dt), dL_dJ=to_dev(gJ, dt), I_rays=I)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "f64" else 2e-5
    for got, want, name in zip(outs, (oc, oS, oIb, oIt), ("chi", "S", "Ib", "It")):
        got = got.cpu().numpy()
        e = normerr(got, want)
        msg = f"  d{name}: normwise {e:.2e}"
        if prec == "f64":
            # element by element too, over every entry above 1e-6 of the largest
            # (smaller ones are sums of terms that cancel to below the rounding of
            # their parts)
            big = np.abs(want) > 1e-6 * np.max(np.abs(want))
            ee = float(np.max(np.abs(got[big] - want[big]) / np.abs(want[big]), initial=0.0))
            msg += f", element-wise {ee:.2e} over {int(big.sum())} of {big.size} entries"
            assert ee <= 1e-10, name
        flush(msg)
        assert e <= tol, name
    G.close()


def test_ray_groups_and_recompute_agree(v, ctx, case):
    flush("vjp ray groups")
    atm, g, dirs, w, sel = case
    nl = 8
    lam = np.linspace(500e-9, 700e-9, nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    rng = np.random.default_rng(2)
    gI = to_dev(rng.standard_normal((len(dirs), g.n, nl)), torch.float64)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    c_d, S_d = to_dev(chi, torch.float64), to_dev(S, torch.float64)
    J = torch.empty_like(c_d)
    I = torch.empty((len(dirs), g.n, nl), dtype=torch.float64, device="cuda:0")
    v.formal_solution(G, c_d, S_d, J, I_rays=I)
    ref = [t.cpu().numpy() for t in v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, I_rays=I)]
    for group, keep in ((5, True), (5, False), (1, False), (24, False)):
        got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, I_rays=I if keep else None, ray_group=group)
        for a, b in zip(got, ref):
            assert normerr(a.cpu().numpy(), b) <= 1e-14, (group, keep)
    # the interleaved record copy of the forward sweeps leaves the reverse sweep
    # as it is (ray groups sum over rays in another order, hence the tolerance)
    G.tune(v.VRT_TUNE_INTERLEAVE, 1)
    for group, keep in ((0, True), (0, False), (24, False), (5, False)):
        got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, I_rays=I if keep else None, ray_group=group)
        for a, b in zip(got, ref):
            if group % 24 == 0:
                assert np.array_equal(a.cpu().numpy(), b), ("interleaved", group, keep)
            else:
                assert normerr(a.cpu().numpy(), b) <= 1e-14, ("interleaved", group, keep)
    G.close()


@pytest.mark.parametrize("nl", [8, 64])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_persistent_reverse_matches_level_steps(v, ctx, case, nl, prec):
    """The persistent reverse sweep performs the level-step reverse sweep's
    arithmetic per record, so its adjoints are bit-identical, for all rays at
    once and for ray groups, with kept and recomputed forward intensities;
    a spin bound of zero polls reports a timeout and the next call is correct."""
    flush(f"persistent reverse nl={nl} {prec}")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    chi = chi * np.random.default_rng(nl + 7).uniform(0.5, 2.0, (1, nl))
    rng = np.random.default_rng(3)
    dt = torch.float64 if prec == "f64" else torch.float32
    gI = to_dev(rng.standard_normal((len(dirs), g.n, nl)), dt)
    gJ = to_dev(rng.standard_normal((g.n, nl)), dt)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    c_d, S_d = to_dev(chi, dt), to_dev(S, dt)
    J = torch.empty_like(c_d)
    I = torch.empty((len(dirs), g.n, nl), dtype=dt, device="cuda:0")
    v.formal_solution(G, c_d, S_d, J, I_rays=I)
    for group, keep in ((0, True), (5, False), (24, False)):
        ref = [t.cpu().numpy() for t in v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ,
                                                               I_rays=I if keep else None, ray_group=group)]
        G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 1)
        got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ, I_rays=I if keep else None, ray_group=group)
        G.device_status()
        G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 0)
        for a, b in zip(got, ref):
            assert np.array_equal(a.cpu().numpy(), b), (group, keep)
    G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 1)
    G.tune(v.VRT_TUNE_SPIN_CAP, 0)
    v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, I_rays=I)
    with pytest.raises(v.VrtError) as e:
        G.device_status()
    assert e.value.status == v.VRT_E_TIMEOUT
    G.tune(v.VRT_TUNE_SPIN_CAP, 1 << 22)
    got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ, I_rays=I)
    G.device_status()
    G.tune(v.VRT_TUNE_REVERSE_PERSISTENT, 0)
    ref = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ, I_rays=I)
    for a, b in zip(got, ref):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    G.close()


@pytest.mark.parametrize("nl", [8, 64])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_level_chunk_checkpoints_are_bit_identical(v, ctx, case, nl, prec):
    """Per-level-chunk checkpoints of the recomputed forward intensities (the
    frontier rows a later chunk reads, and each chunk recomputed just before
    its reverse steps) give the same bits as keeping every row, for chunks of
    one step, a few steps and more steps than the sweep has, with and without
    ray groups; the autograd misfit gradient is the same with and without."""
    flush(f"vjp checkpoints nl={nl} {prec}")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    chi = chi * np.random.default_rng(nl + 11).uniform(0.5, 2.0, (1, nl))
    rng = np.random.default_rng(13)
    dt = torch.float64 if prec == "f64" else torch.float32
    gI = to_dev(rng.standard_normal((len(dirs), g.n, nl)), dt)
    gJ = to_dev(rng.standard_normal((g.n, nl)), dt)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    levels = G.info()["max_levels"]
    c_d, S_d = to_dev(chi, dt), to_dev(S, dt)
    for group in (0, 5):
        ref = [t.cpu().numpy() for t in v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ, ray_group=group)]
        for k in (1, 3, 7, levels - 1, levels, 10 * levels):
            got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, dL_dJ=gJ, ray_group=group, checkpoint_levels=k)
            for a, b in zip(got, ref):
                assert np.array_equal(a.cpu().numpy(), b), (group, k)
    full = v.formal_solution_vjp_scratch(G, dt, nl, keep_intensities=False, ray_group=5)
    kept = v.formal_solution_vjp_scratch(G, dt, nl, keep_intensities=True, ray_group=5)
    part = v.formal_solution_vjp_scratch(G, dt, nl, keep_intensities=False, ray_group=5, checkpoint_levels=7)
    flush(f"  scratch bytes: kept {kept}, recomputed {full}, checkpointed every 7 steps {part}")
    # the checkpointed rows (beyond the plan's 16 bytes per sweep record) are
    # fewer than a ray group's full rows
    plan = 16 * len(dirs) * g.n
    assert 0 < part - kept - plan < full - kept
    # the record order re-packs the sweep records (and so the plan)
    G.tune(v.VRT_TUNE_RECORD_ORDER, 0)
    G.set_rays(dirs, w)
    ref = [t.cpu().numpy() for t in v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, ray_group=3)]
    got = v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, ray_group=3, checkpoint_levels=4)
    for a, b in zip(got, ref):
        assert np.array_equal(a.cpu().numpy(), b)
    with pytest.raises(v.VrtError):
        v.formal_solution_vjp(G, c_d, S_d, dL_dI=gI, checkpoint_levels=-1)
    # through autograd, with the forward intensities dropped after the forward pass
    T0, r0 = to_dev(atm.T, torch.float64), to_dev(atm.rho, torch.float64)
    grads = []
    for k in (0, 5):
        T = T0.clone().requires_grad_(True)
        rho = r0.clone().requires_grad_(True)
        v.lte_emergent(T, rho, G, lam, atm.kappa0, dtype=dt, keep_intensities=False, ray_group=4,
                       checkpoint_levels=k).double().pow(2).sum().backward()
        grads.append((T.grad.cpu().numpy(), rho.grad.cpu().numpy()))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    G.close()


@pytest.mark.parametrize("fwd", ["f64 persistent", "f32 graph"])
def test_reverse_sweep_on_the_last_solutions_rows(v, ctx, case, fwd):
    """The reverse sweep on the last formal solution's rows kept by the library
    (sign-encoded rows of the FP64 persistent sweep, or plain FP32 rows),
    converted to the sweep's precision, equals the reverse sweep handed the
    same rows bit for bit. Any later solve, or a solution into caller rows,
    makes the solution unusable (VRT_E_STATE)."""
    flush(f"vjp on the last solution ({fwd})")
    atm, g, dirs, w, sel = case
    nl = 8
    lam = np.linspace(500e-9, 700e-9, nl)
    chi, S = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    R = len(dirs)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    dt = torch.float64 if fwd.startswith("f64") else torch.float32
    mode = v.VRT_EXEC_PERSISTENT if "persistent" in fwd else v.VRT_EXEC_GRAPH
    c_f, s_f = to_dev(chi, dt), to_dev(S, dt)
    J = torch.empty_like(c_f)
    I_ref = torch.empty((R, g.n, nl), dtype=dt, device="cuda:0")
    v.formal_solution(G, c_f, s_f, J, I_rays=I_ref, exec_mode=v.VRT_EXEC_GRAPH)
    v.formal_solution(G, c_f, s_f, J, exec_mode=mode)
    sid = G.solution_id()
    f32 = torch.float32
    c32, s32 = to_dev(chi, f32), to_dev(S, f32)
    gI = to_dev(np.random.default_rng(3).standard_normal((R, g.n, nl)), f32)
    got = v.formal_solution_vjp_last(G, sid, c32, s32, dL_dI=gI)
    want = v.formal_solution_vjp(G, c32, s32, dL_dI=gI, I_rays=I_ref.to(f32).contiguous())
    G.device_status()
    for a, b in zip(got, want):
        assert torch.equal(a, b)
    # a ray group at a time, from the same converted rows
    got2 = v.formal_solution_vjp_last(G, sid, c32, s32, dL_dI=gI, ray_group=5)
    want2 = v.formal_solution_vjp(G, c32, s32, dL_dI=gI, I_rays=I_ref.to(f32).contiguous(), ray_group=5)
    for a, b in zip(got2, want2):
        assert torch.equal(a, b)
    v.formal_solution(G, c_f, s_f, J, exec_mode=mode)
    with pytest.raises(v.VrtError) as e:
        v.formal_solution_vjp_last(G, sid, c32, s32, dL_dI=gI)
    assert e.value.status == v.VRT_E_STATE
    v.formal_solution(G, c_f, s_f, J, I_rays=I_ref, exec_mode=mode)
    with pytest.raises(v.VrtError) as e:
        v.formal_solution_vjp_last(G, G.solution_id(), c32, s32, dL_dI=gI)
    assert e.value.status == v.VRT_E_STATE
    G.close()


def test_autograd_reuses_the_forward_rows_or_recomputes(v, ctx, case):
    """The differentiable emergent intensity takes its backward pass's forward
    rows from its own FP64 forward solution, and recomputes them in FP32 when
    the grid has solved again in between; the two gradients agree to the
    single-precision rounding of the rows."""
    flush("autograd reuse or recompute")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, 4)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    off, _ = G.emergent_index()
    cvec = to_dev(np.random.default_rng(8).standard_normal((int(off[-1]), len(lam))), torch.float64)
    grads = []
    for intervene in (False, True):
        T = to_dev(atm.T, torch.float64).requires_grad_(True)
        rho = to_dev(atm.rho, torch.float64).requires_grad_(True)
        L = (v.lte_emergent(T, rho, G, lam, atm.kappa0, dtype=torch.float32).double() * cvec).sum()
        if intervene:
            x = torch.ones((g.n, 2), dtype=torch.float32, device="cuda:0")
            v.formal_solution(G, x, x, torch.empty_like(x))
        L.backward()
        grads.append((T.grad.cpu().numpy(), rho.grad.cpu().numpy()))
    for a, b in zip(grads[0], grads[1]):
        assert normerr(a, b) <= 1e-5
    G.close()


def test_lte_chain_rule_matches_oracle(v, ctx, case):
    flush("lte vjp")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, 5)
    rng = np.random.default_rng(3)
    gc, gS, gIb = (rng.standard_normal((g.n, 5)) for _ in range(3))
    oT, orho = oracle.lte_vjp(lam, atm.kappa0, atm.T, atm.rho, gc, gS, gIb)
    G = v.Grid.from_synth(ctx, g)
    d = torch.float64
    gT, gr = v.lte_continuum_vjp(G, lam, atm.kappa0, to_dev(atm.T, d), to_dev(atm.rho, d), to_dev(gc, d),
                                 to_dev(gS, d), to_dev(gIb, d))
    torch.cuda.synchronize()
    assert normerr(gT.cpu().numpy(), oT) <= 1e-13
    assert normerr(gr.cpu().numpy(), orho) <= 1e-13
    G.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_autograd_misfit_gradient(v, ctx, case, prec):
    """L = sum (I_emergent - I_target)^2 with the target from a 2% perturbed temperature."""
    flush(f"autograd misfit {prec}")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, 4)
    Tt = atm.T * (1 + 0.02 * np.random.default_rng(11).standard_normal(g.n))
    _, _, _, It = oracle.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, Tt, atm.rho)
    em = oracle.emergent_sites(g, dirs)
    target = {r: It[r, em[r]] for r in range(len(dirs)) if dirs[r, 2] > 0}
    Lo, oT, orho, _ = oracle.emergent_loss(g, dirs, w, sel, lam, atm.kappa0, atm.T, atm.rho, target)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    dt = torch.float64 if prec == "f64" else torch.float32
    off, sites = G.emergent_index()
    tgt = np.zeros((int(off[-1]), len(lam)))
    mask = np.zeros((int(off[-1]), 1))
    for r in range(len(dirs)):
        if dirs[r, 2] > 0:
            tgt[off[r]:off[r + 1]] = target[r]
            mask[off[r]:off[r + 1]] = 1.0
    T = to_dev(atm.T, torch.float64).requires_grad_(True)
    rho = to_dev(atm.rho, torch.float64).requires_grad_(True)
    I_em = v.lte_emergent(T, rho, G, lam, atm.kappa0, dtype=dt)
    L = (((I_em.double() - to_dev(tgt, torch.float64)) ** 2) * to_dev(mask, torch.float64)).sum()
    L.backward()
    tol = 1e-10 if prec == "f64" else 1e-4
    assert abs(L.item() - Lo) <= (1e-12 if prec == "f64" else 1e-5) * abs(Lo)
    eT = normerr(T.grad.cpu().numpy(), oT)
    er = normerr(rho.grad.cpu().numpy(), orho)
    flush(f"  dL/dT err {eT:.2e}  dL/drho err {er:.2e}")
    assert eT <= tol and er <= tol
    G.close()


def test_adjoint_matches_central_differences_on_gpu(v, ctx, case):
    """The FP32-sweep adjoint agrees with central differences of the FP64 GPU
    forward within 1e-4 at sites where the perturbation is resolvable."""
    flush("adjoint vs FD")
    atm, g, dirs, w, sel = case
    lam = np.linspace(500e-9, 700e-9, 4)
    G = v.Grid.from_synth(ctx, g)
    G.set_rays(dirs, w)
    off, _ = G.emergent_index()
    rng = np.random.default_rng(5)
    cvec = to_dev(rng.standard_normal((int(off[-1]), len(lam))), torch.float64)

    def L_of(T, rho, dt):
        with torch.no_grad():
            return float((v.lte_emergent(T, rho, G, lam, atm.kappa0, dtype=dt).double() * cvec).sum().item())

    T = to_dev(atm.T, torch.float64).requires_grad_(True)
    rho = to_dev(atm.rho, torch.float64).requires_grad_(True)
    (v.lte_emergent(T, rho, G, lam, atm.kappa0, dtype=torch.float32).double() * cvec).sum().backward()
    gT = T.grad.cpu().numpy()
    gr = rho.grad.cpu().numpy()
    chi, _ = oracle.lte(lam, atm.kappa0, atm.T, atm.rho)
    thick = np.nonzero((chi[:, 0] * 1e5 > 1e-2) & (np.abs(gT) > 1e-3 * np.max(np.abs(gT))))[0]
    for i in np.random.default_rng(6).choice(thick, 8, replace=False):
        for base, grad, name in ((atm.T, gT, "T"), (atm.rho, gr, "rho")):
            h = 1e-5 * base[i]
            vals = []
            for sgn in (1, -1):
                a = base.copy()
                a[i] += sgn * h
                Tt = to_dev(a if name == "T" else atm.T, torch.float64)
                rr = to_dev(a if name == "rho" else atm.rho, torch.float64)
                vals.append(L_of(Tt, rr, torch.float64))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-4 * max(abs(fd), 1e-3 * np.max(np.abs(grad))), (name, i, fd, grad[i])
    G.close()
