"""Upwind selection (Sect. 2.5, Eq. 5-6) and per-ray level schedules.

Pins: a hand-built neighbour star with angles worked out by hand; a brute
force that ranks candidate Delaunay lines by their angle to the ray
(arccos of the normalised dot product, i.e. the paper's "smallest angle"
wording rather than the oracle's squared-cosine key); levels from a memoised
longest-path recursion; and invariance of everything under a relabelling of
the sites.
"""

import numpy as np
import pytest

import synth


def _star_grid():
    # site 0 at the origin with six neighbours below it and one above; box tall enough
    P = np.array([
        [0.0, 0.0, 0.0],
        [0.0, 0.0, -1.0],            # straight below
        [1.0, 0.0, -1.0],            # 45 deg off vertical, towards +x
        [-1.0, 0.0, -1.0],           # 45 deg towards -x
        [0.0, 2.0, -1.0],            # further off
        [0.3, 0.1, -2.0],            # nearly vertical, long
        [0.5, 0.5, 0.0],             # same height: never a candidate
        [0.0, 0.0, 1.0],             # above
    ])
    n = len(P)
    nbrs = {0: [1, 2, 3, 4, 5, 6, 7]}
    for k in range(1, n):
        nbrs[k] = [0]
    ptr = np.zeros(n + 1, np.int64)
    idx = []
    for i in range(n):
        idx += nbrs[i]
        ptr[i + 1] = len(idx)
    g = synth.VoronoiGrid(xyz=P, nbr_ptr=ptr, nbr_idx=np.array(idx, np.int32),
                          nbr_shift=np.zeros((len(idx), 2), np.int8),
                          wall=np.array([0, 1, 1, 1, 1, 1, 3, 2], np.uint8),
                          lo=np.array([-5, -5, -3.0]), hi=np.array([5, 5, 2.0]), periodic_xy=False)
    return g


def test_hand_built_star(orc):
    g = _star_grid()
    # ray 30 degrees from vertical in the x-z plane
    th = np.deg2rad(30.0)
    n = np.array([[np.sin(th), 0.0, np.cos(th)]])
    sel = orc.select(g, n, r_exp=7.0)
    # angles to the lines from neighbours 1..5 into site 0 (d = r_0 - r_k):
    #  k=1: d=(0,0,1) -> 30 deg; k=2: d=(-1,0,1) -> 75 deg (n.d<0? sin30*-1+cos30 = 0.366 >0)
    #  k=3: d=(1,0,1) -> 15 deg; k=4: d=(0,-2,1) -> cos = cos30/sqrt5 -> 67.2 deg
    #  k=5: d=(-0.3,-0.1,2) -> cos = (-0.15+1.732)/2.025 -> 38.6 deg
    assert sel.k1[0, 0] == 3 and sel.k2[0, 0] == 1
    v1 = np.cos(np.deg2rad(15.0))
    v2 = np.cos(np.deg2rad(30.0))
    assert abs(sel.w1[0, 0] - v1**7 / (v1**7 + v2**7)) < 1e-14
    assert abs(sel.ds1[0, 0] - np.sqrt(2.0)) < 1e-15 and abs(sel.ds2[0, 0] - 1.0) < 1e-15
    # the bottom-wall sites are boundary sites of the upward ray
    assert np.all(sel.k1[0, 1:6] == -1)
    # the top site (wall bit 1 only) takes site 0 as its single candidate
    assert sel.k1[0, 7] == 0 and sel.k2[0, 7] == -1 and sel.w1[0, 7] == 1.0
    # a downward ray: site 0 has one z-upwind neighbour (7) with n.d > 0 iff the ray points down
    sel_d = orc.select(g, -n, r_exp=7.0)
    assert sel_d.k1[0, 0] == 7 and sel_d.k2[0, 0] == -1


def test_fallback_when_no_forward_line(orc):
    g = _star_grid()
    # a very shallow ray pointing towards -x: only neighbour 2 lies below with n.d<=0? use the key rule
    n = np.array([[-np.sqrt(1 - 1e-4), 0.0, 1e-2]])
    sel = orc.select(g, n)
    # candidates with n.d > 0: d=(1,0,1) (k=3 side) has n.d = -0.99995+0.01 < 0; d=(0,0,1): 0.01 > 0
    # so k=1 is a candidate (dot 0.01) and k=2, d=(-1,0,1): n.d = 0.99995+0.01 > 0
    assert sel.k1[0, 0] == 2 and sel.k2[0, 0] in (1, 5)


def _brute_select(g, dirs, r_exp=7.0):
    n = g.n
    R = len(dirs)
    L = g.hi - g.lo
    out = {}
    for r in range(R):
        nv = dirs[r]
        sig = 1 if nv[2] > 0 else -1
        upbit = 1 if nv[2] > 0 else 2
        for i in range(n):
            if g.wall[i] & upbit:
                out[r, i] = (-1, -1, 1.0)
                continue
            cands = []
            zup = []
            for e in range(g.nbr_ptr[i], g.nbr_ptr[i + 1]):
                k = int(g.nbr_idx[e])
                d = g.xyz[i] - g.xyz[k] - np.array([g.nbr_shift[e, 0] * L[0], g.nbr_shift[e, 1] * L[1], 0.0])
                if sig * d[2] <= 0:
                    continue
                cosang = float(np.dot(nv, d) / np.linalg.norm(d))
                ang = np.arccos(np.clip(cosang, -1, 1))
                zup.append((ang, k, cosang))
                if cosang > 0:
                    cands.append((ang, k, cosang))
            cands.sort()
            zup.sort()
            if len(cands) >= 2:
                a, b = cands[0], cands[1]
                w = a[2] ** r_exp / (a[2] ** r_exp + b[2] ** r_exp)
                out[r, i] = (a[1], b[1], w)
            elif len(cands) == 1:
                out[r, i] = (cands[0][1], -1, 1.0)
            else:
                out[r, i] = (zup[0][1], -1, 1.0)
    return out


@pytest.fixture(scope="module")
def small_grid():
    atm = synth.make_atmosphere(600, seed=99)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    return g


def test_selection_matches_angle_brute_force(orc, small_grid):
    g = small_grid
    dirs, _ = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    bf = _brute_select(g, dirs)
    for (r, i), (a, b, w) in bf.items():
        assert sel.k1[r, i] == a and sel.k2[r, i] == b, (r, i)
        assert abs(sel.w1[r, i] - w) <= 1e-12, (r, i)


def _memo_levels(k1, k2):
    n = len(k1)
    lev = np.full(n, -1, np.int64)

    import sys
    sys.setrecursionlimit(10000)

    def f(i):
        if lev[i] >= 0:
            return lev[i]
        if k1[i] < 0:
            lev[i] = 0
        else:
            m = f(k1[i])
            if k2[i] >= 0:
                m = max(m, f(k2[i]))
            lev[i] = m + 1
        return lev[i]

    for i in range(n):
        f(i)
    return lev


def test_levels_match_longest_path_recursion(orc, small_grid):
    g = small_grid
    dirs, _ = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    level, order, ptrs, nlev = orc.levels(g, dirs, sel)
    for r in range(len(dirs)):
        want = _memo_levels(sel.k1[r], sel.k2[r])
        assert np.array_equal(level[r], want)
        assert nlev[r] == want.max() + 1
        ord_want = np.lexsort((np.arange(g.n), want))
        assert np.array_equal(order[r], ord_want)
        assert np.array_equal(ptrs[r], np.searchsorted(want[ord_want], np.arange(nlev[r] + 1)))
        # boundary sites are exactly the level-0 sites and the wall sites on the upwind side
        bit = 1 if dirs[r, 2] > 0 else 2
        assert np.array_equal(level[r] == 0, (g.wall & bit) > 0)


def test_relabelling_invariance(orc, small_grid):
    g = small_grid
    dirs, _ = synth.gauss_legendre_quadrature()
    rng = np.random.default_rng(4)
    perm = rng.permutation(g.n)         # new index of old site i is inv[i]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    xyz2 = g.xyz[perm]
    rows = []
    for new_i in range(g.n):
        old_i = perm[new_i]
        s, e = g.nbr_ptr[old_i], g.nbr_ptr[old_i + 1]
        rows.append((inv[g.nbr_idx[s:e]], g.nbr_shift[s:e]))
    ptr2 = np.zeros(g.n + 1, np.int64)
    ptr2[1:] = np.cumsum([len(r[0]) for r in rows])
    g2 = synth.VoronoiGrid(xyz=xyz2, nbr_ptr=ptr2, nbr_idx=np.concatenate([r[0] for r in rows]).astype(np.int32),
                           nbr_shift=np.concatenate([r[1] for r in rows]).astype(np.int8), wall=g.wall[perm],
                           lo=g.lo, hi=g.hi, periodic_xy=True)
    s1 = orc.select(g, dirs)
    s2 = orc.select(g2, dirs)
    l1, _, _, n1 = orc.levels(g, dirs, s1)
    l2, _, _, n2 = orc.levels(g2, dirs, s2)
    assert np.array_equal(n1, n2)
    for r in range(len(dirs)):
        k1_map = np.where(s1.k1[r, perm] >= 0, inv[np.maximum(s1.k1[r, perm], 0)], -1)
        k2_map = np.where(s1.k2[r, perm] >= 0, inv[np.maximum(s1.k2[r, perm], 0)], -1)
        assert np.array_equal(s2.k1[r], k1_map)
        assert np.array_equal(s2.k2[r], k2_map)
        assert np.array_equal(s2.w1[r], s1.w1[r, perm])
        assert np.array_equal(l2[r], l1[r, perm])


def test_lattice_rays_follow_vertical_lines(orc):
    # on a lattice the only strictly-lower neighbour is straight below, so every
    # upward ray is carried along vertical lines with weight 1 (reading R1/R5)
    z = np.array([0.0, 0.5, 0.7, 1.5])
    g = synth.lattice_grid(3, 3, z)
    dirs, _ = synth.gauss_legendre_quadrature()
    sel = orc.select(g, dirs)
    for r in range(len(dirs)):
        for i in range(g.n):
            iz = i // 9
            up = dirs[r, 2] > 0
            if (up and iz == 0) or (not up and iz == 3):
                assert sel.k1[r, i] == -1
            else:
                assert sel.k1[r, i] == (i - 9 if up else i + 9)
                assert sel.k2[r, i] == -1 and sel.w1[r, i] == 1.0
                assert sel.ds1[r, i] == abs(z[iz] - z[iz - 1 if up else iz + 1])
