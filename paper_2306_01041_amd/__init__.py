"""MI355X (gfx950) formal solution of the radiative transfer equation on irregular
(Voronoi) and regular grids, after Udnaes & Pereira (2023, arXiv:2306.01041).

The compute path is the HIP library ``libvrt.so`` (C ABI in ``include/vrt.h``);
``paper_2306_01041_amd.vrt`` is its ctypes binding. Importing the binding raises
ImportError when the library has not been built; there is no CPU fallback.
"""

__version__ = "0.1.0"


def load():
    """Import and return the binding module (raises if libvrt.so is missing)."""
    from . import vrt

    return vrt
