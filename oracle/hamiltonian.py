"""Matrix-free Kohn-Sham Hamiltonian on a uniform 3-D grid (oracle; test infrastructure only).

Section 2.1 of the paper: H is never formed; its action on a block of
orbitals is the sum of three parts,

  (1) the finite-difference Laplacian stencil,  T x = -1/2 Lap_FD x,
  (2) the effective potential multiplied pointwise, Veff * x,
  (3) the nonlocal Kleinman-Bylander projectors of every atom J applied as a
      dense product on the grid points S_J the atom's projectors touch,
        (V_nl x)[S_J] += chi_J Gamma_J (chi_J^T x[S_J]) dV,
      with Gamma_J = diag(gamma_J) (energies in Ha) and dV = hx*hy*hz.

A problem is any object with attributes ``n`` (Nx, Ny, Nz), ``h``, ``bc``
(0 periodic / 1 Dirichlet per direction), ``fd_order``, ``veff`` (Nd,),
``supp_ptr``, ``supp_idx``, ``nproj``, ``chi`` (per atom, column-major
n_J x np_J) and ``gamma``.  Grid point (x, y, z) has linear index
x + Nx*(y + Ny*z); an orbital block is an (Nd, Ns) float64 array here.
"""
from __future__ import annotations

import numpy as np

from .fd import second_derivative_weights

# numpy axis of each Cartesian direction for a (Nz, Ny, Nx, ...) array
_AXIS = {0: 2, 1: 1, 2: 0}


def _shift(u: np.ndarray, p: int, direction: int, periodic: bool) -> np.ndarray:
    """Return v with v[..i..] = u[..i+p..] along ``direction``; zero ghosts if not periodic."""
    ax = _AXIS[direction]
    if periodic:
        return np.roll(u, -p, axis=ax)
    n = u.shape[ax]
    v = np.zeros_like(u)
    if abs(p) >= n:
        return v
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if p > 0:
        src[ax] = slice(p, n)
        dst[ax] = slice(0, n - p)
    else:
        src[ax] = slice(0, n + p)
        dst[ax] = slice(-p, n)
    v[tuple(dst)] = u[tuple(src)]
    return v


def kinetic(prob, x: np.ndarray) -> np.ndarray:
    """T x = -1/2 sum_d h_d^-2 sum_{p=-r..r} w_|p| x[i + p e_d] (Section 2.1, stencil bullet)."""
    nx, ny, nz = prob.n
    w = second_derivative_weights(prob.fd_order)
    r = len(w) - 1
    ns = x.shape[1]
    u = x.reshape(nz, ny, nx, ns)
    lap = np.zeros_like(u)
    for d in range(3):
        inv_h2 = 1.0 / (prob.h[d] * prob.h[d])
        periodic = prob.bc[d] == 0
        lap += (w[0] * inv_h2) * u
        for p in range(1, r + 1):
            lap += (w[p] * inv_h2) * (_shift(u, p, d, periodic) + _shift(u, -p, d, periodic))
    return (-0.5 * lap).reshape(-1, ns)


def local_potential(prob, x: np.ndarray) -> np.ndarray:
    """Veff multiplied pointwise into every column (Section 2.1, second bullet)."""
    return prob.veff[:, None] * x


def atom_blocks(prob):
    """Yield (support indices, chi_J (n_J x np_J), gamma_J) for every atom."""
    coff = 0
    goff = 0
    for J in range(len(prob.nproj)):
        lo, hi = int(prob.supp_ptr[J]), int(prob.supp_ptr[J + 1])
        nj = hi - lo
        npj = int(prob.nproj[J])
        idx = np.asarray(prob.supp_idx[lo:hi], dtype=np.int64)
        chi = np.asarray(prob.chi[coff:coff + nj * npj]).reshape(npj, nj).T
        gam = np.asarray(prob.gamma[goff:goff + npj])
        coff += nj * npj
        goff += npj
        yield idx, chi, gam


def nonlocal_potential(prob, x: np.ndarray) -> np.ndarray:
    """sum_J chi_J Gamma_J chi_J^T x[S_J] dV, scattered back to S_J (Section 2.1, third bullet)."""
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    y = np.zeros_like(x)
    for idx, chi, gam in atom_blocks(prob):
        coeff = dv * (chi.T @ x[idx, :])          # np_J x Ns
        y[idx, :] += chi @ (gam[:, None] * coeff)
    return y


def apply_h(prob, x: np.ndarray) -> np.ndarray:
    """H x for an (Nd, Ns) block: kinetic + local + nonlocal parts."""
    x = np.asarray(x, dtype=np.float64)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[:, None]
    y = kinetic(prob, x) + local_potential(prob, x) + nonlocal_potential(prob, x)
    return y[:, 0] if squeeze else y


def dense_h(prob) -> np.ndarray:
    """The full Nd x Nd matrix of H, built by applying H to every unit vector (tiny grids only)."""
    nd = int(prob.n[0] * prob.n[1] * prob.n[2])
    if nd > 4096:
        raise ValueError("dense_h is for tiny grids only")
    return apply_h(prob, np.eye(nd))
