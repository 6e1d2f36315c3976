"""CheFSI at a Bloch wavevector k with complex arithmetic (oracle; test infrastructure only).

The paper runs Gamma-point (and isolated) systems in real arithmetic and every other
Brillouin-zone sample in complex FP64 (Sec. 2, the paragraph on the GPU strategy); H in
Alg. 1 is the Hamiltonian of one Bloch wavevector.  Here H_k acts on Bloch-periodic
orbitals, psi(r + L_d e_d) = exp(i k_d L_d) psi(r) in every periodic direction d:

  kinetic    the FD Laplacian of Sec. 2.1 whose ghost values across a periodic face carry
             the phase exp(+-i k_d L_d) (Dirichlet directions keep zero ghosts, k_d unused);
  local      Veff multiplied pointwise;
  nonlocal   each projector is its Bloch sum  chi~_J(r) = sum_T chi_J(r - R_J - T) exp(i k.T).
             With the truncation radius below half the cell, a support point of atom J sees
             one image, T = m L (m in Z^3 per point: the point lies at R_J + m L + offset), so
             chi~_J(point) = chi_J(offset) exp(i k.(m L)); then
             V_nl psi = sum_J chi~_J Gamma_J (chi~_J^H psi[S_J]) dV.

The CheFSI step is Alg. 1 with conjugate transposes: Hs = X~^H H X~, Ms = X~^H X~,
Hs Z = Ms Z D (Hermitian-definite), X = X~ Z.  The filter scalars are real, as before.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .fd import second_derivative_weights
from .hamiltonian import atom_blocks

_AXIS = {0: 2, 1: 1, 2: 0}


def cell_phases(prob, k):
    """exp(i k_d L_d) per direction (1 in Dirichlet directions), L_d = N_d h_d."""
    out = []
    for d in range(3):
        if prob.bc[d] == 0:
            out.append(np.exp(1j * k[d] * prob.n[d] * prob.h[d]))
        else:
            out.append(1.0 + 0.0j)
    return out


def _bloch_shift(u, p, d, periodic, phase):
    """v[..i..] = psi(i + p) along direction d for a Bloch-periodic psi given on the cell:
    points past the upper face are psi(i + p - N) exp(i k L), below the lower face
    psi(i + p + N) exp(-i k L); zero ghosts when not periodic."""
    ax = _AXIS[d]
    n = u.shape[ax]
    idx = np.arange(n) + p
    wraps = np.floor_divide(idx, n)          # cell translations crossed by i + p
    v = np.take(u, np.mod(idx, n), axis=ax)
    if periodic:
        fac = np.power(complex(phase), wraps)
    else:
        fac = np.where(wraps == 0, 1.0, 0.0).astype(complex)
    shape = [1] * u.ndim
    shape[ax] = n
    return v * fac.reshape(shape)


def kinetic_k(prob, x, k):
    """T_k x = -1/2 sum_d h_d^-2 sum_{p=-r..r} w_|p| x~(i + p e_d), x~ the Bloch extension."""
    nx, ny, nz = prob.n
    w = second_derivative_weights(prob.fd_order)
    r = len(w) - 1
    ns = x.shape[1]
    u = np.asarray(x, dtype=complex).reshape(nz, ny, nx, ns)
    ph = cell_phases(prob, k)
    lap = np.zeros_like(u)
    for d in range(3):
        inv_h2 = 1.0 / (prob.h[d] * prob.h[d])
        periodic = prob.bc[d] == 0
        lap += (w[0] * inv_h2) * u
        for p in range(1, r + 1):
            lap += (w[p] * inv_h2) * (_bloch_shift(u, p, d, periodic, ph[d]) +
                                      _bloch_shift(u, -p, d, periodic, ph[d]))
    return (-0.5 * lap).reshape(-1, ns)


def projector_blocks_k(prob, img, k):
    """Yield (support indices, chi~_J (n_J x np_J complex), gamma_J) per atom; img is the
    (sum n_J, 3) integer image m of every support point."""
    L = [prob.n[d] * prob.h[d] for d in range(3)]
    kl = np.array([k[d] * L[d] if prob.bc[d] == 0 else 0.0 for d in range(3)])
    off = 0
    for idx, chi, gam in atom_blocks(prob):
        m = np.asarray(img[off:off + len(idx)], dtype=float)
        off += len(idx)
        phase = np.exp(1j * (m @ kl))
        yield idx, chi * phase[:, None], gam


def nonlocal_k(prob, img, k, x):
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    y = np.zeros(x.shape, dtype=complex)
    for idx, chi, gam in projector_blocks_k(prob, img, k):
        coeff = dv * (chi.conj().T @ x[idx, :])
        y[idx, :] += chi @ (gam[:, None] * coeff)
    return y


def apply_h_k(prob, img, k, x):
    """H_k x for an (Nd, Ns) complex block."""
    x = np.asarray(x, dtype=complex)
    squeeze = x.ndim == 1
    if squeeze:
        x = x[:, None]
    y = kinetic_k(prob, x, k) + prob.veff[:, None] * x + nonlocal_k(prob, img, k, x)
    return y[:, 0] if squeeze else y


def dense_h_k(prob, img, k):
    nd = int(prob.n[0] * prob.n[1] * prob.n[2])
    if nd > 4096:
        raise ValueError("dense_h_k is for tiny grids only")
    return apply_h_k(prob, img, k, np.eye(nd, dtype=complex))


def chebyshev_filter_k(prob, img, k, x, degree, lam_lo, lam_cut, lam_hi):
    """The scaled three-term Chebyshev filter of Alg. 1 (real scalars) on a complex block."""
    c = 0.5 * (lam_hi + lam_cut)
    e = 0.5 * (lam_hi - lam_cut)
    y_prev = np.array(x, dtype=complex)
    if degree == 0:
        return y_prev
    s1 = e / (lam_lo - c)
    s = s1
    y = (s1 / e) * (apply_h_k(prob, img, k, y_prev) - c * y_prev)
    for _ in range(1, degree):
        s_next = 1.0 / (2.0 / s1 - s)
        y_next = (2.0 * s_next / e) * (apply_h_k(prob, img, k, y) - c * y) - (s * s_next) * y_prev
        y_prev, y = y, y_next
        s = s_next
    return y


def project_k(prob, img, k, xf):
    """Hs = X~^H (H_k X~), Ms = X~^H X~, each made exactly Hermitian by (A + A^H) / 2."""
    yf = apply_h_k(prob, img, k, xf)
    hs = xf.conj().T @ yf
    ms = xf.conj().T @ xf
    return 0.5 * (hs + hs.conj().T), 0.5 * (ms + ms.conj().T)


def chefsi_step_k(prob, img, k, x, degree, lam_lo, lam_cut, lam_hi):
    """One complex CheFSI step: (ascending Ritz values, rotated block)."""
    xf = chebyshev_filter_k(prob, img, k, x, degree, lam_lo, lam_cut, lam_hi)
    hs, ms = project_k(prob, img, k, xf)
    d, z = scipy.linalg.eigh(hs, ms, type=1, driver="gvd")
    return d, xf @ z
