"""Nonlocal (Kleinman-Bylander) part of the Hellmann-Feynman atomic forces (oracle; test
infrastructure only).

Sec. 2 of the paper: the stencil and projector routines of the filter are reused for the
nonlocal components of the forces and stresses, whose key kernels are the gradient
operator applied to the Kohn-Sham orbitals followed by the nonlocal projectors applied to
the result.  For real orbitals psi_n with occupations g_n the nonlocal energy is

    E_nl = sum_n g_n sum_{J,a} gamma_Ja (dV chi_Ja^T psi_n)^2 .

Moving atom J moves chi_Ja(r - R_J); integration by parts (periodic directions, or
orbitals that vanish at a Dirichlet boundary) turns d(chi^T psi)/dR_J into chi^T grad psi:

    F_J = -dE_nl/dR_J = -2 sum_n g_n sum_a gamma_Ja (dV chi_Ja^T psi_n) (dV chi_Ja^T grad psi_n).

grad is the central finite-difference first derivative of the same order 2r as the
Laplacian, with the closed-form weights (limit of Lagrange interpolation on 2r+1 nodes)

    d psi / dx_d (i) ~ (1/h_d) sum_{p=1..r} c_p (psi[i + p e_d] - psi[i - p e_d]),
    c_p = (-1)^(p+1) (r!)^2 / (p (r-p)! (r+p)!).
"""
from __future__ import annotations

import math

import numpy as np

from .hamiltonian import _shift, atom_blocks


def first_derivative_weights(order: int) -> np.ndarray:
    """c_1..c_r (index 0 unused, zero) of the central first-derivative stencil of even ``order``."""
    if order < 2 or order % 2:
        raise ValueError("finite-difference order must be even and >= 2")
    r = order // 2
    c = np.zeros(r + 1)
    for p in range(1, r + 1):
        c[p] = (-1.0) ** (p + 1) * math.factorial(r) ** 2 / (p * math.factorial(r - p) * math.factorial(r + p))
    return c


def gradient(prob, x: np.ndarray, direction: int) -> np.ndarray:
    """d x / d x_direction for an (Nd, Ns) block (periodic wrap or zero ghosts)."""
    nx, ny, nz = prob.n
    c = first_derivative_weights(prob.fd_order)
    ns = x.shape[1]
    u = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx, ns)
    periodic = prob.bc[direction] == 0
    g = np.zeros_like(u)
    for p in range(1, len(c)):
        g += c[p] * (_shift(u, p, direction, periodic) - _shift(u, -p, direction, periodic))
    return (g / prob.h[direction]).reshape(-1, ns)


def nonlocal_forces(prob, psi: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """(n_atoms, 3) nonlocal forces for orbitals psi (Nd x Ns) with occupations occ (Ns)."""
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    psi = np.asarray(psi, dtype=np.float64)
    grads = [gradient(prob, psi, d) for d in range(3)]
    forces = []
    for idx, chi, gam in atom_blocks(prob):
        a = dv * (chi.T @ psi[idx, :])                     # np_J x Ns
        f = np.zeros(3)
        for d in range(3):
            b = dv * (chi.T @ grads[d][idx, :])
            f[d] = -2.0 * float(np.sum(gam[:, None] * occ[None, :] * a * b))
        forces.append(f)
    return np.array(forces).reshape(-1, 3)


def nonlocal_energy(prob, psi: np.ndarray, occ: np.ndarray) -> float:
    """E_nl = sum_n g_n sum_{J,a} gamma_Ja (dV chi_Ja^T psi_n)^2."""
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    e = 0.0
    for idx, chi, gam in atom_blocks(prob):
        a = dv * (chi.T @ psi[idx, :])
        e += float(np.sum(gam[:, None] * occ[None, :] * a * a))
    return e


def nonlocal_stress(prob, psi: np.ndarray, occ: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """Nonlocal (Kleinman-Bylander) component of the stress (3 x 3, Ha / bohr^3), the other
    force-like quantity Sec. 2 evaluates with the gradient of the orbitals followed by the
    projectors.  Under a homogeneous strain eps the cell, the grid and the atoms move with
    (1 + eps), dV takes the factor det(1 + eps), the grid values of a normalised orbital the
    factor det^-1/2, and every projector is sampled at the strained displacement
    (1 + eps) d, d = r_i - R_J.  So

        E_nl(eps) = det(1 + eps) sum_n g_n sum_{J,a} gamma_Ja (dV sum_i chi_Ja((1 + eps) d_i) psi_n,i)^2,

    and d chi((1 + eps) d) / d eps_ab = (d_a chi)(d) d_b.  Integrating by parts over the
    support (chi vanishes on its edge) turns sum_i (d_a chi) d_b psi into
    -sum_i chi (delta_ab psi + d_b d_a psi), so sigma_ab = (1 / Omega) dE_nl / d eps_ab is

        sigma_ab = -(1 / Omega) [delta_ab E_nl + 2 sum_n g_n sum_{J,a} gamma_Ja alpha_Ja,n beta_Ja,n;ab],
        alpha = dV chi^T psi_n,   beta_ab = dV sum_i chi(i) d_b(i) (d psi_n / dx_a)(i),

    with the FD gradient of the Laplacian's order (``gradient``) and Omega = Nd dV.
    ``disp`` is (sum n_J, 3): d for every support point, in the order of ``supp_idx``."""
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    psi = np.asarray(psi, dtype=np.float64)
    disp = np.asarray(disp, dtype=np.float64).reshape(-1, 3)
    omega = psi.shape[0] * dv
    grads = [gradient(prob, psi, a) for a in range(3)]
    e_nl = nonlocal_energy(prob, psi, occ)
    s = np.zeros((3, 3))
    for J, (idx, chi, gam) in enumerate(atom_blocks(prob)):
        dJ = disp[int(prob.supp_ptr[J]):int(prob.supp_ptr[J + 1])]
        alpha = dv * (chi.T @ psi[idx, :])                     # np_J x Ns
        for a in range(3):
            for b in range(3):
                beta = dv * ((chi * dJ[:, b:b + 1]).T @ grads[a][idx, :])
                s[a, b] += 2.0 * float(np.sum(gam[:, None] * occ[None, :] * alpha * beta))
    return -(np.eye(3) * e_nl + s) / omega


def kinetic_stress(prob, psi: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """Electronic kinetic-energy component of the stress (3 x 3, Ha / bohr^3) from the FD
    gradient of the orbitals (Sec. 2 reuses that gradient for it):

        sigma_ab = -(1 / Omega) sum_n g_n dV sum_i (d psi_n / dx_a)(i) (d psi_n / dx_b)(i),

    Omega = Nd dV the cell volume; real orbitals."""
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    psi = np.asarray(psi, dtype=np.float64)
    omega = psi.shape[0] * dv
    g = [gradient(prob, psi, d) for d in range(3)]
    s = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            s[a, b] = -dv / omega * float(np.sum(occ[None, :] * g[a] * g[b]))
    return s
