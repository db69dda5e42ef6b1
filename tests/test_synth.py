"""Input generators: quadrature, atmosphere recipe, Voronoi neighbour lists and lattices.

The Voronoi adjacency is pinned by an independent brute-force definition (a
linear programme per site pair: do the two cells share a face of positive area
inside the box?), by the mean degree of Poisson-Voronoi cells, 2 + 48 pi^2/35
= 15.5355 (the paper quotes 15.54, Sect. 2.5), and by exact lattice results.
"""

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import linprog

import synth
from synth.atmosphere import MM, KM


def test_quadrature_moments():
    dirs, w = synth.gauss_legendre_quadrature()
    assert dirs.shape == (24, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-15)
    # GL(3) on [0,1] integrates mu^2 exactly: angle mean of mu^2 is 1/3
    assert abs(np.sum(w * dirs[:, 2] ** 2) - 1.0 / 3.0) < 1e-15
    assert np.allclose(np.sum(w[:, None] * dirs, axis=0), 0.0, atol=1e-15)
    mus = np.unique(np.round(np.abs(dirs[:, 2]), 12))
    assert np.allclose(mus, [0.5 - np.sqrt(0.15), 0.5, 0.5 + np.sqrt(0.15)], atol=1e-12)
    # no ray along the x or y axis
    assert np.all(np.abs(dirs[:, 0]) > 0.1) and np.all(np.abs(dirs[:, 1]) > 0.1)


def test_temperature_and_density_recipe():
    assert abs(synth.T0_of_z(-0.5 * MM) - 6500.0) < 1.0
    assert abs(synth.T0_of_z(0.5 * MM) - 4241.0) < 1.0
    assert abs(synth.T0_of_z(2.5 * MM) - 4200.0) < 1e-9
    assert abs(synth.rho_of_z(0.0) - 3e-4) < 1e-18
    assert abs(synth.rho_of_z(150 * KM) - 3e-4 / np.e) < 1e-15


def test_kappa0_normalises_tau_to_one_at_z0():
    kappa0, _, _ = synth.kappa0_and_density()
    box = synth.BoxSpec()

    def g(z):
        return kappa0 * synth.rho_of_z(z) ** 2 * synth.T0_of_z(z) ** 9

    inside, _ = quad(g, 0.0, box.hi[2], limit=400, epsabs=0, epsrel=1e-12)
    tail = g(box.hi[2]) * 150 * KM / 2.0
    assert abs(inside + tail - 1.0) < 1e-7
    # chi(0) of the recipe
    assert 1.5e-5 < g(0.0) < 1.8e-5


def test_horizontal_field_statistics():
    f = synth.horizontal_field(3)
    assert abs(f.mean()) < 1e-12 and abs(f.std() - 1.0) < 1e-12
    # correlation at one correlation length ~ exp(-1/2) (loose: finite box)
    lag = int(round(256 / 6.0))
    c = np.mean(f * np.roll(f, lag, axis=0))
    assert 0.35 < c < 0.85


def test_rejection_sampling_follows_target_density():
    _, zt, ft = synth.kappa0_and_density()
    xyz = synth.sample_sites(200000, seed=5)
    box = synth.BoxSpec()
    assert np.all(xyz >= np.asarray(box.lo)) and np.all(xyz <= np.asarray(box.hi))
    hist, edges = np.histogram(xyz[:, 2], bins=30, range=(box.lo[2], box.hi[2]))
    mids = 0.5 * (edges[1:] + edges[:-1])
    expect = np.interp(mids, zt, ft)
    expect = expect / expect.sum() * hist.sum()
    chi2 = np.sum((hist - expect) ** 2 / expect)
    assert chi2 < 80  # 29 dof


def _face_lp(P, i, k_img, others, lo, hi, clip_xy):
    """Largest slack t with a point x on the bisector of P[i] and k_img, strictly
    closer to both than to every point in ``others`` and inside the box by t."""
    a = P[i]
    b = k_img
    A_ub, b_ub = [], []
    for c in others:
        A_ub.append(np.r_[2 * (c - a), 1.0])
        b_ub.append(c @ c - a @ a)
    dims = [0, 1, 2] if clip_xy else [2]
    for d in dims:
        e = np.zeros(4); e[d] = -1; e[3] = 1; A_ub.append(e); b_ub.append(-lo[d])
        e = np.zeros(4); e[d] = 1; e[3] = 1; A_ub.append(e); b_ub.append(hi[d])
    A_eq = [np.r_[2 * (b - a), 0.0]]
    b_eq = [b @ b - a @ a]
    res = linprog(c=[0, 0, 0, -1], A_ub=np.array(A_ub), b_ub=np.array(b_ub), A_eq=np.array(A_eq),
                  b_eq=np.array(b_eq), bounds=[(None, None)] * 3 + [(None, 1.0)], method="highs")
    return -res.fun if res.status == 0 else -np.inf


def _wall_lp(P, i, others, lo, hi, zwall, clip_xy):
    """Largest slack t with a point of cell i on the plane z = zwall."""
    a = P[i]
    A_ub, b_ub = [], []
    for c in others:
        A_ub.append(np.r_[2 * (c - a), 1.0])
        b_ub.append(c @ c - a @ a)
    if clip_xy:
        for d in (0, 1):
            e = np.zeros(4); e[d] = -1; e[3] = 1; A_ub.append(e); b_ub.append(-lo[d])
            e = np.zeros(4); e[d] = 1; e[3] = 1; A_ub.append(e); b_ub.append(hi[d])
    A_eq = [np.array([0, 0, 1.0, 0])]
    res = linprog(c=[0, 0, 0, -1], A_ub=np.array(A_ub), b_ub=np.array(b_ub), A_eq=np.array(A_eq),
                  b_eq=[zwall], bounds=[(None, None)] * 3 + [(None, 1.0)], method="highs")
    return -res.fun if res.status == 0 else -np.inf


@pytest.mark.parametrize("periodic", [False, True])
def test_voronoi_adjacency_brute_force(periodic):
    rng = np.random.default_rng(11 + periodic)
    n = 24 if periodic else 40
    lo = np.zeros(3)
    hi = np.array([1.0, 1.2, 0.9])
    P = lo + rng.random((n, 3)) * (hi - lo)
    g = synth.voronoi_neighbours(P, lo, hi, periodic_xy=periodic, margin_spacings=10.0)
    assert synth.check_symmetric(g)
    L = hi - lo
    shifts = [(sx, sy) for sx in (-1, 0, 1) for sy in (-1, 0, 1)] if periodic else [(0, 0)]
    imgs = {s: P + np.array([s[0] * L[0], s[1] * L[1], 0.0]) for s in shifts}
    got = set()
    for i in range(n):
        for e in range(g.nbr_ptr[i], g.nbr_ptr[i + 1]):
            got.add((i, int(g.nbr_idx[e]), int(g.nbr_shift[e, 0]), int(g.nbr_shift[e, 1])))
    want = set()
    for i in range(n):
        for s in shifts:
            for k in range(n):
                if k == i and s == (0, 0):
                    continue
                others = [imgs[t][j] for t in shifts for j in range(n) if not (t == s and j == k)
                          and not (t == (0, 0) and j == i)]
                if _face_lp(P, i, imgs[s][k], others, lo, hi, clip_xy=not periodic) > 1e-9:
                    want.add((i, k, s[0], s[1]))
    assert got == want
    for i in range(n):
        others = [imgs[t][j] for t in shifts for j in range(n) if not (t == (0, 0) and j == i)]
        bot = _wall_lp(P, i, others, lo, hi, lo[2], clip_xy=not periodic) > 1e-9
        top = _wall_lp(P, i, others, lo, hi, hi[2], clip_xy=not periodic) > 1e-9
        assert bool(g.wall[i] & 1) == bot and bool(g.wall[i] & 2) == top, i


def test_voronoi_adjacency_does_not_depend_on_margin():
    atm = synth.make_atmosphere(3000, seed=17)
    g1 = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi, margin_spacings=4.0)
    g2 = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi, margin_spacings=8.0)
    assert np.array_equal(g1.nbr_ptr, g2.nbr_ptr)
    assert np.array_equal(g1.nbr_idx, g2.nbr_idx)
    assert np.array_equal(g1.nbr_shift, g2.nbr_shift)
    assert np.array_equal(g1.wall, g2.wall)


def test_poisson_voronoi_mean_degree():
    # interior cells of a uniform random box: theory 2 + 48 pi^2 / 35 (paper: 15.54)
    rng = np.random.default_rng(2)
    P = rng.random((30000, 3))
    g = synth.voronoi_neighbours(P, [0, 0, 0], [1, 1, 1])
    far = (P[:, 2] > 0.2) & (P[:, 2] < 0.8)
    deg = g.degrees()[far]
    theory = 2.0 + 48.0 * np.pi**2 / 35.0
    assert abs(theory - 15.5355) < 1e-4
    sem = deg.std() / np.sqrt(len(deg))
    assert abs(deg.mean() - theory) < 4 * sem


def test_recipe_grid_degree_and_walls():
    atm = synth.make_atmosphere(16384, seed=1041)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    assert synth.check_symmetric(g)
    assert 14.8 < g.m / g.n < 15.5
    assert 700 < np.count_nonzero(g.wall & 1) < 1100
    assert 700 < np.count_nonzero(g.wall & 2) < 1100
    # every non-wall cell has a neighbour strictly below and strictly above
    src = np.repeat(np.arange(g.n), np.diff(g.nbr_ptr))
    dz = g.xyz[src, 2] - g.xyz[g.nbr_idx, 2]
    has_below = np.zeros(g.n, bool); has_below[src[dz > 0]] = True
    has_above = np.zeros(g.n, bool); has_above[src[dz < 0]] = True
    assert np.all(has_below | (g.wall & 1 > 0))
    assert np.all(has_above | (g.wall & 2 > 0))


def test_lattice_neighbours():
    z = np.array([0.0, 0.3, 1.0, 1.1, 2.0])
    g = synth.lattice_grid(4, 3, z, dx=0.5, dy=0.7)
    assert synth.check_symmetric(g)
    deg = g.degrees()
    nz = len(z)
    iz = np.arange(g.n) // 12
    assert np.all(deg[(iz > 0) & (iz < nz - 1)] == 6)
    assert np.all(deg[(iz == 0) | (iz == nz - 1)] == 5)
    assert np.all((g.wall & 1) == (iz == 0))
    assert np.all(((g.wall >> 1) & 1) == (iz == nz - 1))
    # a 2-wide periodic direction gives the same neighbour twice with different shifts
    g2 = synth.lattice_grid(2, 2, z)
    assert synth.check_symmetric(g2)
    assert np.all(g2.degrees()[6:14] == 6)


def test_concat_grids_is_a_disjoint_union():
    gs = []
    for n, seed in ((60, 3), (200, 4)):
        atm = synth.make_atmosphere(n, seed=seed)
        gs.append(synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi))
    gs.append(gs[0])
    U, off = synth.concat_grids(gs)
    assert list(off) == [0, gs[0].n, gs[0].n + gs[1].n, U.n] and U.n == sum(g.n for g in gs)
    assert U.m == sum(g.m for g in gs)
    assert synth.check_symmetric(U)
    for a, g in enumerate(gs):
        for i in range(g.n):
            j = off[a] + i
            nb = U.nbr_idx[U.nbr_ptr[j] : U.nbr_ptr[j + 1]]
            assert np.array_equal(nb, g.nbr_idx[g.nbr_ptr[i] : g.nbr_ptr[i + 1]] + off[a])
            assert np.array_equal(U.nbr_shift[U.nbr_ptr[j] : U.nbr_ptr[j + 1]], g.nbr_shift[g.nbr_ptr[i] : g.nbr_ptr[i + 1]])
        assert np.array_equal(U.xyz[off[a] : off[a + 1]], g.xyz) and np.array_equal(U.wall[off[a] : off[a + 1]], g.wall)


def test_batch_sizes_are_seeded_and_in_range():
    s = synth.batch_sizes(48, 32768, 524288, seed=1041)
    assert s == synth.batch_sizes(48, 32768, 524288, seed=1041)
    assert len(s) == 48 and min(s) >= 32768 and max(s) <= 524288
    # log-uniform: about half below the geometric mean of the bounds
    assert 14 <= sum(x < np.sqrt(32768 * 524288) for x in s) <= 34


@pytest.mark.parametrize("name", ["alpha_c", "log_nhii", "log_nh_t"])
def test_design_densities_are_sampled_in_proportion(name):
    """Rejection sampling (Sect. 2.4) reproduces the target density: the
    height histogram of the accepted sites matches the x-y integral of f."""
    from synth import design

    box = synth.BoxSpec()
    n = 200000
    xyz = design.sample_sites_density(n, 11, name)
    assert xyz.shape == (n, 3)
    assert np.all(xyz >= np.asarray(box.lo)) and np.all(xyz <= np.asarray(box.hi))
    edges = np.linspace(box.lo[2], box.hi[2], 13)
    got = np.histogram(xyz[:, 2], edges)[0] / n
    rng = np.random.default_rng(12)
    probe = np.asarray(box.lo) + rng.random((1 << 21, 3)) * box.L
    f = design.target_density(name, probe)
    want = np.histogram(probe[:, 2], edges, weights=f)[0]
    want /= want.sum()
    big = want > 0.01
    assert np.all(np.abs(got[big] - want[big]) <= 0.05 * want[big] + 0.002)


def test_design_densities_order_the_heights():
    """The line-oriented density puts more sites high in the box than the
    continuum extinction (which piles them at the bottom)."""
    from synth import design

    zc = np.median(design.sample_sites_density(20000, 3, "alpha_c")[:, 2])
    zl = np.median(design.sample_sites_density(20000, 3, "log_nh_t")[:, 2])
    assert zc < 0.0 < zl


def test_locality_order_numbers_sites_by_slab_then_morton():
    """Generated sites come numbered slab by slab (one mean spacing thick,
    bottom to top) and along the Morton curve of (x, y) inside a slab; the set
    of sites is the accepted sample itself, only renumbered."""
    box = synth.BoxSpec()
    raw = synth.sample_sites(5000, seed=44, ordered=False)
    xyz = synth.sample_sites(5000, seed=44)
    perm = synth.locality_order(raw, box)
    assert np.array_equal(np.sort(perm), np.arange(len(raw)))
    assert np.array_equal(xyz, raw[perm])
    lo, L = np.asarray(box.lo), box.L
    h = float(np.prod(L) / len(xyz)) ** (1 / 3)
    slab = np.floor((xyz[:, 2] - lo[2]) / h).astype(np.int64)
    assert np.all(np.diff(slab) >= 0)
    q = np.clip(np.floor((xyz[:, :2] - lo[:2]) / L[:2] * 65536.0), 0, 65535).astype(np.int64)

    def morton(ix, iy):
        m = 0
        for b in range(16):
            m |= ((ix >> b) & 1) << (2 * b) | ((iy >> b) & 1) << (2 * b + 1)
        return m

    keys = [(int(s_), morton(int(a), int(b))) for s_, (a, b) in zip(slab, q)]
    assert keys == sorted(keys)
    # neighbours in the numbering are neighbours in space: the mean distance
    # between consecutive sites is a few spacings, not a box size
    step = np.linalg.norm(np.diff(xyz, axis=0), axis=1)
    assert np.median(step) < 3 * h
