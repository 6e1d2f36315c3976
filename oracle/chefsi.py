"""Algorithm 1 of the paper (CheFSI-based partial diagonalisation) in plain FP64 (oracle; test infrastructure only).

One CheFSI step on an orbital block X (Nd x Ns):

  Filtering        X~ = p_m((H - cI)/e) X,  c = (lam_hi + lam_cut)/2,
                   e = (lam_hi - lam_cut)/2                     (Alg. 1, Filtering)
  Projection       H~ = X~^T (H X~),  M~ = X~^T X~              (Alg. 1, Projection; Sec. 2.2)
  Diagonalisation  H~ Z~ = M~ Z~ D~                              (Alg. 1, Diagonalization; Sec. 2.3)
  Rotation         X = X~ Z~                                     (Alg. 1, Rotation; Sec. 2.4)

The paper names lam_hi the largest eigenvalue of H and lam_cut the filter
cutoff but does not say how they are obtained; the bounds used here are
listed in ``spectral_bounds``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .fd import second_derivative_weights
from .hamiltonian import apply_h, atom_blocks


# ---------------------------------------------------------------------------
# Filtering (Algorithm 1, Filtering block; Section 2.1)
# ---------------------------------------------------------------------------
def chebyshev_filter_unscaled(prob, x, degree, lam_cut, lam_hi):
    """p_m((H - cI)/e) X by the three-term Chebyshev recurrence, exactly as Alg. 1 writes it.

    T_0(L) X = X, T_1(L) X = L X, T_{k+1}(L) X = 2 L T_k(L) X - T_{k-1}(L) X with L = (H - cI)/e.
    """
    c = 0.5 * (lam_hi + lam_cut)
    e = 0.5 * (lam_hi - lam_cut)
    t_prev = np.array(x, dtype=np.float64)
    if degree == 0:
        return t_prev
    t_cur = (apply_h(prob, t_prev) - c * t_prev) / e
    for _ in range(1, degree):
        t_next = 2.0 * (apply_h(prob, t_cur) - c * t_cur) / e - t_prev
        t_prev, t_cur = t_cur, t_next
    return t_cur


def chebyshev_filter(prob, x, degree, lam_lo, lam_cut, lam_hi):
    """Scaled Chebyshev filter: p_m((H - cI)/e) X / p_m((lam_lo - c)/e).

    Same polynomial as Alg. 1; dividing by the scalar p_m(l0), l0 = (lam_lo - c)/e,
    keeps the iterates O(1).  With rho_k = T_k(l0) and s_k = rho_{k-1}/rho_k the
    recurrence T_{k+1} = 2 L T_k - T_{k-1} becomes
        Y_1     = (s_1 / e) (H - cI) X,                 s_1 = e / (lam_lo - c),
        Y_{k+1} = (2 s_{k+1} / e) (H - cI) Y_k - s_k s_{k+1} Y_{k-1},
        1 / s_{k+1} = 2 / s_1 - s_k.
    """
    c = 0.5 * (lam_hi + lam_cut)
    e = 0.5 * (lam_hi - lam_cut)
    y_prev = np.array(x, dtype=np.float64)
    if degree == 0:
        return y_prev
    s1 = e / (lam_lo - c)
    s = s1
    y = (s1 / e) * (apply_h(prob, y_prev) - c * y_prev)
    for _ in range(1, degree):
        s_next = 1.0 / (2.0 / s1 - s)
        y_next = (2.0 * s_next / e) * (apply_h(prob, y) - c * y) - (s * s_next) * y_prev
        y_prev, y = y, y_next
        s = s_next
    return y


def filter_scalars(degree, lam_lo, lam_cut, lam_hi):
    """(c, e, [s_1 .. s_m]) of the scaled filter, for checking a kernel's coefficients."""
    c = 0.5 * (lam_hi + lam_cut)
    e = 0.5 * (lam_hi - lam_cut)
    s1 = e / (lam_lo - c)
    ss = [s1]
    for _ in range(1, degree):
        ss.append(1.0 / (2.0 / s1 - ss[-1]))
    return c, e, ss


def chebyshev_t(m: int, t: float) -> float:
    """T_m(t) from its trigonometric / hyperbolic closed form (no recurrence)."""
    if abs(t) <= 1.0:
        return math.cos(m * math.acos(t))
    if t > 1.0:
        return math.cosh(m * math.acosh(t))
    return (-1.0) ** m * math.cosh(m * math.acosh(-t))


# ---------------------------------------------------------------------------
# Projection, diagonalisation, rotation (Algorithm 1; Sections 2.2-2.4)
# ---------------------------------------------------------------------------
def project(prob, xf):
    """H~ = X~^T Y~ with Y~ = H X~, and M~ = X~^T X~ (Alg. 1, Projection), symmetrised."""
    yf = apply_h(prob, xf)
    hs = xf.T @ yf
    ms = xf.T @ xf
    return 0.5 * (hs + hs.T), 0.5 * (ms + ms.T)


def diagonalize(hs, ms):
    """Solve H~ Z~ = M~ Z~ D~ (Alg. 1, Diagonalization; Sec. 2.3 uses the dense dsygvd routine).

    Returns (D ascending, Z) with Z^T M~ Z = I.
    """
    d, z = scipy.linalg.eigh(hs, ms, type=1, driver="gvd")
    return d, z


def diagonalize_by_cholesky(hs, ms):
    """Same problem through Cholesky: M = L L^T, C = L^-1 H L^-T = W D W^T, Z = L^-T W."""
    lo = np.linalg.cholesky(ms)
    a = scipy.linalg.solve_triangular(lo, hs, lower=True)
    c = scipy.linalg.solve_triangular(lo, a.T, lower=True).T
    c = 0.5 * (c + c.T)
    d, w = np.linalg.eigh(c)
    z = scipy.linalg.solve_triangular(lo.T, w, lower=False)
    return d, z


def rotate(xf, z):
    """X = X~ Z~ (Alg. 1, Rotation)."""
    return xf @ z


def chefsi_step(prob, x, degree, lam_lo, lam_cut, lam_hi):
    """One CheFSI step (filter, project, diagonalise, rotate).  Returns (ritz values D, new X)."""
    xf = chebyshev_filter(prob, x, degree, lam_lo, lam_cut, lam_hi)
    hs, ms = project(prob, xf)
    d, z = diagonalize(hs, ms)
    return d, rotate(xf, z)


def chefsi(prob, x0, degree, n_iter, lam_lo, lam_cut, lam_hi, callback=None):
    """n_iter CheFSI steps with the bounds update lam_lo <- D_1, lam_cut <- D_Ns (lam_hi fixed).

    The update rule is this implementation's reading; the paper only names the
    cutoff and the largest eigenvalue.
    """
    x = np.array(x0, dtype=np.float64)
    d = None
    for it in range(n_iter):
        d, x = chefsi_step(prob, x, degree, lam_lo, lam_cut, lam_hi)
        if callback is not None:
            callback(it, d, x, lam_lo, lam_cut)
        lam_lo, lam_cut = float(d[0]), float(d[-1])
    return d, x


# ---------------------------------------------------------------------------
# Spectral bounds for the filter (reading: the paper does not say how they are found)
# ---------------------------------------------------------------------------
def spectral_bounds(prob):
    """(lam_lo, lam_cut, lam_hi) for the first step.

    lam_hi: Gershgorin / Weyl upper bound on the largest eigenvalue of H,
        1/2 sum_d sum_{|p|<=r} |w_p| / h_d^2 + max Veff
        + max_i sum_{(J,a) touching i} |gamma_Ja| |chi_Ja(i)| ||chi_Ja||_1 dV.
    lam_lo: min Veff, a lower bound on the spectrum when every gamma >= 0 (the
        kinetic and nonlocal parts are then positive semidefinite); otherwise
        the nonlocal bound is subtracted as well.
    lam_cut: lam_lo + 0.1 (lam_hi - lam_lo).
    """
    w = second_derivative_weights(prob.fd_order)
    s = abs(w[0]) + 2.0 * np.abs(w[1:]).sum()
    kin = 0.5 * sum(s / (prob.h[d] * prob.h[d]) for d in range(3))
    dv = prob.h[0] * prob.h[1] * prob.h[2]
    nd = int(prob.n[0] * prob.n[1] * prob.n[2])
    row = np.zeros(nd)
    any_negative = False
    for idx, chi, gam in atom_blocks(prob):
        for a in range(chi.shape[1]):
            row[idx] += abs(gam[a]) * np.abs(chi[:, a]) * np.abs(chi[:, a]).sum() * dv
            any_negative = any_negative or gam[a] < 0
    nl = float(row.max()) if nd else 0.0
    lam_hi = kin + float(np.max(prob.veff)) + nl
    lam_lo = float(np.min(prob.veff)) - (nl if any_negative else 0.0)
    lam_cut = lam_lo + 0.1 * (lam_hi - lam_lo)
    return lam_lo, lam_cut, lam_hi


# ---------------------------------------------------------------------------
# Comparison metrics (rotation- and sign-invariant)
# ---------------------------------------------------------------------------
def subspace_residual(x_ref, x_test, k):
    """sin of the largest principal angle between span(x_ref[:, :k]) and span(x_test[:, :k])."""
    q_ref, _ = np.linalg.qr(x_ref[:, :k])
    q_test, _ = np.linalg.qr(x_test[:, :k])
    r = q_test - q_ref @ (q_ref.T @ q_test)
    return float(np.linalg.norm(r, 2))


def residual_norms(prob, x, d):
    """max_j ||H x_j - d_j x_j|| / ||x_j|| over the columns of x."""
    hx = apply_h(prob, x)
    res = hx - x * d[None, :]
    return np.linalg.norm(res, axis=0) / np.linalg.norm(x, axis=0)


def gap_index(d, k_max, min_gap=1e-3):
    """Largest k <= k_max with d[k] - d[k-1] >= min_gap (a block boundary between Ritz clusters)."""
    for k in range(min(k_max, len(d) - 1), 0, -1):
        if d[k] - d[k - 1] >= min_gap:
            return k
    return 0
