"""Voronoi neighbour lists (the grid data model of Sect. 2.4) built from a Delaunay triangulation.

The paper takes cell neighbours from voro++ in a box container that is
periodic in x and y and clipped by walls at the bottom and top. That library is
not available; the same adjacency is obtained from Qhull's Delaunay
triangulation (scipy) of the sites plus

* periodic images in x and y within a margin of the box, and
* mirror images across the bottom and top z-walls within a margin.

For a point set symmetric under reflection in a wall plane, the Voronoi cell of
a site restricted to its own side is exactly the cell clipped by the wall, and
the face shared with its own mirror image is the wall itself. Hence two
original sites are neighbours of the clipped diagram iff they are Delaunay
neighbours of the augmented set, and a cell touches a wall iff the site is a
Delaunay neighbour of its own mirror. Edges to other mirror images bound faces
outside the box and are dropped.

Output layout (caller site order): CSR ``nbr_ptr`` int64 [n+1], ``nbr_idx``
int32 [m], ``nbr_shift`` int8 [m, 2] and ``wall`` uint8 [n] (bit 0: the cell
touches the bottom wall z = lo, bit 1: the top wall z = hi). The neighbour
entry (k, sx, sy) of site i means that the image of site k adjacent to i sits
at r_k + (sx * Lx, sy * Ly, 0). Rows are sorted by (k, sx, sy).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class VoronoiGrid:
    xyz: np.ndarray        # [n, 3] float64
    nbr_ptr: np.ndarray    # [n + 1] int64
    nbr_idx: np.ndarray    # [m] int32
    nbr_shift: np.ndarray  # [m, 2] int8
    wall: np.ndarray       # [n] uint8
    lo: np.ndarray         # [3] float64
    hi: np.ndarray         # [3] float64
    periodic_xy: bool = True

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def m(self) -> int:
        return int(self.nbr_idx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.nbr_ptr)


def _csr_from_edges(n, src, dst, sx, sy):
    key = np.lexsort((sy, sx, dst, src))
    src, dst, sx, sy = src[key], dst[key], sx[key], sy[key]
    # drop duplicates
    if len(src):
        keep = np.ones(len(src), dtype=bool)
        keep[1:] = (src[1:] != src[:-1]) | (dst[1:] != dst[:-1]) | (sx[1:] != sx[:-1]) | (sy[1:] != sy[:-1])
        src, dst, sx, sy = src[keep], dst[keep], sx[keep], sy[keep]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, src + 1, 1)
    ptr = np.cumsum(ptr)
    shift = np.stack([sx, sy], axis=1).astype(np.int8)
    return ptr, dst.astype(np.int32), np.ascontiguousarray(shift)


def voronoi_neighbours(xyz, lo, hi, periodic_xy: bool = True, margin_spacings: float = 4.0) -> VoronoiGrid:
    """Neighbour lists and wall flags of the wall-clipped (and x-y periodic) Voronoi diagram."""
    from scipy.spatial import Delaunay

    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    L = hi - lo
    n = xyz.shape[0]
    h = (np.prod(L) / max(n, 1)) ** (1.0 / 3.0)
    margin = margin_spacings * h

    pts = [xyz]
    src = [np.arange(n, dtype=np.int64)]
    shx = [np.zeros(n, dtype=np.int64)]
    shy = [np.zeros(n, dtype=np.int64)]
    if periodic_xy:
        mx = min(margin, 0.5 * L[0])
        my = min(margin, 0.5 * L[1])
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                if sx == 0 and sy == 0:
                    continue
                p = xyz + np.array([sx * L[0], sy * L[1], 0.0])
                keep = ((p[:, 0] >= lo[0] - mx) & (p[:, 0] <= hi[0] + mx)
                        & (p[:, 1] >= lo[1] - my) & (p[:, 1] <= hi[1] + my))
                idx = np.nonzero(keep)[0]
                pts.append(p[idx])
                src.append(idx)
                shx.append(np.full(len(idx), sx, dtype=np.int64))
                shy.append(np.full(len(idx), sy, dtype=np.int64))
    P = np.concatenate(pts)
    S = np.concatenate(src)
    SX = np.concatenate(shx)
    SY = np.concatenate(shy)
    # 0 real/periodic, 1 bottom mirror, 2 top mirror, 3 mirror across an x or y wall
    kind = np.zeros(len(P), dtype=np.int8)
    if not periodic_xy:
        for ax in (0, 1):
            m = min(margin, 0.5 * L[ax])
            parts = [P]
            meta = [(S, SX, SY, kind)]
            for wall_at in (lo[ax], hi[ax]):
                sel = np.nonzero(np.abs(P[:, ax] - wall_at) <= m)[0]
                Q = P[sel].copy()
                Q[:, ax] = 2.0 * wall_at - Q[:, ax]
                parts.append(Q)
                meta.append((S[sel], SX[sel], SY[sel], np.full(len(sel), 3, np.int8)))
            P = np.concatenate(parts)
            S = np.concatenate([t[0] for t in meta])
            SX = np.concatenate([t[1] for t in meta])
            SY = np.concatenate([t[2] for t in meta])
            kind = np.concatenate([t[3] for t in meta])

    mz = min(margin, 0.5 * L[2])
    bot = np.nonzero(P[:, 2] - lo[2] <= mz)[0]
    top = np.nonzero(hi[2] - P[:, 2] <= mz)[0]
    Pb = P[bot].copy()
    Pb[:, 2] = 2.0 * lo[2] - Pb[:, 2]
    Pt = P[top].copy()
    Pt[:, 2] = 2.0 * hi[2] - Pt[:, 2]
    P = np.concatenate([P, Pb, Pt])
    S = np.concatenate([S, S[bot], S[top]])
    SX = np.concatenate([SX, SX[bot], SX[top]])
    SY = np.concatenate([SY, SY[bot], SY[top]])
    # a z-mirror of an x/y mirror image stays a dropped image (kind 3)
    kb_ = np.where(kind[bot] == 3, 3, 1).astype(np.int8)
    kt_ = np.where(kind[top] == 3, 3, 2).astype(np.int8)
    kind = np.concatenate([kind, kb_, kt_])

    tri = Delaunay(P)
    simp = tri.simplices.astype(np.int64)
    pairs = np.concatenate([simp[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    pairs.sort(axis=1)
    npts = np.int64(len(P))
    keyp = np.unique(pairs[:, 0] * npts + pairs[:, 1])
    a = keyp // npts
    b = keyp % npts
    # keep pairs with at least one original site (index < n); a < b so a is the original one
    sel = a < n
    a, b = a[sel], b[sel]

    wall = np.zeros(n, dtype=np.uint8)
    kb = kind[b]
    own_mirror = ((kb == 1) | (kb == 2)) & (S[b] == a) & (SX[b] == 0) & (SY[b] == 0)
    wall_bits = np.where(kb == 1, 1, 2).astype(np.uint8)
    np.bitwise_or.at(wall, a[own_mirror], wall_bits[own_mirror])

    real = kb == 0
    a, b = a[real], b[real]
    k = S[b]
    sx = SX[b]
    sy = SY[b]
    # each edge in both directions
    e_src = np.concatenate([a, k])
    e_dst = np.concatenate([k, a])
    e_sx = np.concatenate([sx, -sx])
    e_sy = np.concatenate([sy, -sy])
    ptr, idx, shift = _csr_from_edges(n, e_src, e_dst, e_sx, e_sy)
    return VoronoiGrid(xyz=xyz, nbr_ptr=ptr, nbr_idx=idx, nbr_shift=shift, wall=wall,
                       lo=lo, hi=hi, periodic_xy=periodic_xy)


def check_symmetric(g: VoronoiGrid) -> bool:
    """True iff every entry (i -> k, s) has its reverse (k -> i, -s) and no self-loop has zero shift."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.nbr_ptr))
    dst = g.nbr_idx.astype(np.int64)
    sx = g.nbr_shift[:, 0].astype(np.int64)
    sy = g.nbr_shift[:, 1].astype(np.int64)
    if np.any((src == dst) & (sx == 0) & (sy == 0)):
        return False
    f = ((src * n + dst) * 3 + (sx + 1)) * 3 + (sy + 1)
    r = ((dst * n + src) * 3 + (-sx + 1)) * 3 + (-sy + 1)
    return bool(np.array_equal(np.sort(f), np.sort(r)))


def lattice_grid(nx: int, ny: int, z, dx: float = 1.0, dy: float = 1.0, x0: float = 0.0, y0: float = 0.0,
                 periodic_xy: bool = True) -> VoronoiGrid:
    """Voronoi grid of a rectilinear lattice (cells are boxes: six face neighbours).

    Site (ix, iy, iz) has caller index (iz * ny + iy) * nx + ix and position
    (x0 + ix*dx, y0 + iy*dy, z[iz]); z may be non-uniform. Lattice points are
    cospherical, which Qhull cannot triangulate uniquely, so the adjacency is
    written down directly. Wall flags: iz = 0 touches the bottom wall, iz =
    nz - 1 the top wall.
    """
    z = np.asarray(z, dtype=np.float64)
    nz = len(z)
    n = nx * ny * nz
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ix = ix.transpose(2, 1, 0).ravel()
    iy = iy.transpose(2, 1, 0).ravel()
    iz = iz.transpose(2, 1, 0).ravel()
    xyz = np.stack([x0 + ix * dx, y0 + iy * dy, z[iz]], axis=1).astype(np.float64)

    def cid(a, b, c):
        return (c * ny + b) * nx + a

    src, dst, sxs, sys_ = [], [], [], []
    me = np.arange(n, dtype=np.int64)
    for d, (ddx, ddy) in enumerate([(1, 0), (-1, 0), (0, 1), (0, -1)]):
        jx = ix + ddx
        jy = iy + ddy
        sx = np.zeros(n, dtype=np.int64)
        sy = np.zeros(n, dtype=np.int64)
        if periodic_xy:
            sx = np.where(jx >= nx, 1, np.where(jx < 0, -1, 0))
            sy = np.where(jy >= ny, 1, np.where(jy < 0, -1, 0))
            jx = jx % nx
            jy = jy % ny
            ok = np.ones(n, dtype=bool)
        else:
            ok = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny)
        # a periodic direction of length 1 would make a site its own neighbour twice; keep those
        src.append(me[ok]); dst.append(cid(jx, jy, iz)[ok]); sxs.append(sx[ok]); sys_.append(sy[ok])
    for ddz in (1, -1):
        jz = iz + ddz
        ok = (jz >= 0) & (jz < nz)
        src.append(me[ok]); dst.append(cid(ix, iy, jz)[ok])
        sxs.append(np.zeros(ok.sum(), dtype=np.int64)); sys_.append(np.zeros(ok.sum(), dtype=np.int64))
    src = np.concatenate(src); dst = np.concatenate(dst)
    sx = np.concatenate(sxs); sy = np.concatenate(sys_)
    ptr, idx, shift = _csr_from_edges(n, src, dst, sx, sy)
    wall = np.zeros(n, dtype=np.uint8)
    wall[iz == 0] |= 1
    wall[iz == nz - 1] |= 2
    Lz0 = z[0] - (0.5 * (z[1] - z[0]) if nz > 1 else 0.5)
    Lz1 = z[-1] + (0.5 * (z[-1] - z[-2]) if nz > 1 else 0.5)
    lo = np.array([x0 - 0.5 * dx, y0 - 0.5 * dy, Lz0])
    hi = np.array([x0 + (nx - 0.5) * dx, y0 + (ny - 0.5) * dy, Lz1])
    return VoronoiGrid(xyz=xyz, nbr_ptr=ptr, nbr_idx=idx, nbr_shift=shift, wall=wall,
                       lo=lo, hi=hi, periodic_xy=periodic_xy)


def concat_grids(grids):
    """Disjoint union of Voronoi grids that share one box: sites of grid j are
    renumbered by the number of sites before it; no neighbour list crosses
    between grids. Returns (union grid, site offsets [len(grids) + 1])."""
    grids = list(grids)
    if not grids:
        raise ValueError("no grids")
    lo, hi = grids[0].lo, grids[0].hi
    for g in grids:
        if not (np.allclose(g.lo, lo) and np.allclose(g.hi, hi)) or g.periodic_xy != grids[0].periodic_xy:
            raise ValueError("grids of a batch must share one box")
    off = np.zeros(len(grids) + 1, np.int64)
    off[1:] = np.cumsum([g.n for g in grids])
    eoff = np.zeros(len(grids) + 1, np.int64)
    eoff[1:] = np.cumsum([g.m for g in grids])
    xyz = np.concatenate([g.xyz for g in grids])
    ptr = np.concatenate([[0]] + [g.nbr_ptr[1:] + eoff[j] for j, g in enumerate(grids)]).astype(np.int64)
    idx = np.concatenate([g.nbr_idx.astype(np.int64) + off[j] for j, g in enumerate(grids)]).astype(np.int32)
    shift = np.concatenate([g.nbr_shift for g in grids]).astype(np.int8)
    wall = np.concatenate([g.wall for g in grids]).astype(np.uint8)
    return VoronoiGrid(xyz=xyz, nbr_ptr=ptr, nbr_idx=idx, nbr_shift=shift, wall=wall, lo=np.asarray(lo),
                       hi=np.asarray(hi), periodic_xy=grids[0].periodic_xy), off
