"""Helpers shared by the GPU parity tests (not collected by pytest)."""

import numpy as np

import synth


def relerr(a, b):
    """Largest |a - b| / |b| over elements with b != 0; exact zeros must match exactly."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    zero = b == 0
    if zero.any():
        assert np.all(a[zero] == 0), "exact zeros of the oracle are not zero on the GPU"
    nz = ~zero
    if not nz.any():
        return 0.0
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz])))


def recipe_grid(n, seed):
    atm = synth.make_atmosphere(n, seed=seed)
    g = synth.voronoi_neighbours(atm.xyz, atm.box.lo, atm.box.hi)
    return atm, g


def wavelengths(nl, lo=400e-9, hi=900e-9):
    return np.linspace(lo, hi, nl) if nl > 1 else np.array([500e-9])


def to_dev(a, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def flush(msg):
    print(msg, flush=True)
