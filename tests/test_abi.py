"""C-ABI boundary on the CPU: the library loads, exports every function the
header declares, and rejects malformed grids in its host-only validator
(no GPU call is made here)."""

import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def v():
    import paper_2306_01041_amd

    return paper_2306_01041_amd.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "vrt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vrt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    assert "vrt_formal_solution" in names and "vrt_grid_set_rays" in names
    assert len(names) >= 18


def test_library_exports_every_declared_symbol(v):
    import ctypes

    lib = ctypes.CDLL(v.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in v.EXPORTED, name


def test_version_and_status_strings(v):
    assert b"gfx950" in v.vrt_version()
    assert v.vrt_status_string(v.VRT_E_GRID) == b"invalid grid"
    assert v.vrt_status_string(12345) == b"unknown status"


@pytest.fixture(scope="module")
def lattice():
    return synth.lattice_grid(3, 4, [0.0, 1.0, 2.5, 3.0])


def _val(v, g, **over):
    a = dict(n=g.n, xyz=g.xyz, nbr_ptr=g.nbr_ptr, nbr_idx=g.nbr_idx, nbr_shift=g.nbr_shift, wall=g.wall, lo=g.lo,
             hi=g.hi, periodic_xy=g.periodic_xy)
    a.update(over)
    return v.validate_voronoi(**a)


def test_valid_grids_pass(v, lattice):
    assert _val(v, lattice) == (0, "")
    atm = synth.make_atmosphere(800, seed=3)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    assert _val(v, g)[0] == 0


def test_asymmetric_lists_rejected(v, lattice):
    idx = lattice.nbr_idx.copy()
    idx[0] = (idx[0] + 5) % lattice.n
    st, msg = _val(v, lattice, nbr_idx=idx)
    assert st == v.VRT_E_GRID and ("symmetric" in msg or "twice" in msg)


def test_out_of_range_index_rejected(v, lattice):
    idx = lattice.nbr_idx.copy()
    idx[3] = lattice.n + 7
    st, msg = _val(v, lattice, nbr_idx=idx)
    assert st == v.VRT_E_GRID and "out of range" in msg


def test_bad_shift_rejected(v, lattice):
    sh = lattice.nbr_shift.copy()
    sh[0, 0] = 2
    assert _val(v, lattice, nbr_shift=sh)[0] == v.VRT_E_GRID
    assert _val(v, lattice, periodic_xy=False)[0] == v.VRT_E_GRID  # shifts present but not periodic


def test_self_loop_and_bad_ptr_rejected(v):
    xyz = np.array([[0.1, 0.1, 0.1], [0.2, 0.2, 0.2]])
    st, msg = v.validate_voronoi(2, xyz, np.array([0, 1, 2]), np.array([0, 0]), np.zeros((2, 2)), np.array([1, 2]),
                                 np.zeros(3), np.ones(3), True)
    assert st == v.VRT_E_GRID and "itself" in msg
    st, msg = v.validate_voronoi(2, xyz, np.array([0, 2, 1]), np.array([1, 0]), np.zeros((2, 2)), np.array([1, 2]),
                                 np.zeros(3), np.ones(3), True)
    assert st == v.VRT_E_GRID


def test_site_outside_box_and_bad_wall_bits(v, lattice):
    xyz = lattice.xyz.copy()
    xyz[5, 2] = 99.0
    assert _val(v, lattice, xyz=xyz)[0] == v.VRT_E_GRID
    wall = lattice.wall.copy()
    wall[2] = 4
    assert _val(v, lattice, wall=wall)[0] == v.VRT_E_GRID


def test_empty_grid_is_valid(v):
    st, _ = v.validate_voronoi(0, np.zeros((0, 3)), np.array([0]), np.zeros(0), np.zeros((0, 2)), np.zeros(0),
                               np.zeros(3), np.ones(3), True)
    assert st == 0


def test_null_arguments(v):
    st, _ = v.validate_voronoi(3, None, None, None, None, None, np.zeros(3), np.ones(3), True)
    assert st == v.VRT_E_ARG


def test_row_stride_of_strided_views(v):
    """The binding passes chi / S / boundary views with one common row stride
    to vrt_formal_solution_ld: paired slots of one [n][2][nl] array give 2 nl,
    contiguous arrays nl; other element strides, overlapping rows and unequal
    strides are refused before any call."""
    torch = pytest.importorskip("torch")
    n, nl = 5, 6
    f = torch.float32
    cs = torch.zeros((n, 2, nl), dtype=f)
    assert v.row_stride(((cs[:, 0], "chi"), (cs[:, 1], "S"), (None, "I_bottom")), (n, nl), f) == 2 * nl
    a = torch.zeros((n, nl), dtype=f)
    assert v.row_stride(((a, "chi"), (a.clone(), "S")), (n, nl), f) == nl
    wide = torch.zeros((n, nl + 2), dtype=f)
    assert v.row_stride(((wide[:, :nl], "chi"),), (n, nl), f) == nl + 2
    # one site: any stride is a valid layout
    assert v.row_stride(((cs[:1, 0], "chi"),), (1, nl), f) == nl
    with pytest.raises(ValueError, match="adjacent"):
        v.row_stride(((a.t().contiguous().t(), "chi"),), (n, nl), f)
    with pytest.raises(ValueError, match="overlap"):
        v.row_stride(((torch.zeros(n + nl, dtype=f).as_strided((n, nl), (1, 1)), "chi"),), (n, nl), f)
    with pytest.raises(ValueError, match="apart"):
        v.row_stride(((cs[:, 0], "chi"), (a, "S")), (n, nl), f)
    with pytest.raises(ValueError, match="shape"):
        v.row_stride(((a[:, :3], "chi"),), (n, nl), f)
    with pytest.raises(ValueError, match="dtype"):
        v.row_stride(((a.double(), "chi"),), (n, nl), f)
