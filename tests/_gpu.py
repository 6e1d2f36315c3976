"""Helpers for the GPU parity tests: device blocks in the library's layout, and shared tolerances."""
import numpy as np


def torch_mod():
    import torch
    return torch


def dev(x_nd_ns, dtype="float64"):
    """(Nd, ns) host array -> device block (a row-major (ns, Nd) tensor = column-major Nd x ns)."""
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x_nd_ns).T.astype(dtype)))
    return t.cuda()


def host(t):
    """Device block -> (Nd, ns) float64 host array."""
    return t.detach().cpu().numpy().astype(np.float64).T.copy()


def dev_square(a):
    """ns x ns host matrix -> device column-major FP64 (row-major tensor of a^T)."""
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda()


def host_square(t):
    return t.detach().cpu().numpy().T.copy()


def stencil_scale(prob):
    """Sum of the absolute stencil weights times 1/2 h^-2: the size of the terms that cancel in T x."""
    from oracle.chefsi import spectral_bounds
    lo, cut, hi = spectral_bounds(prob)
    return max(abs(lo), abs(hi))
