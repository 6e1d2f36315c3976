"""Estimate of lam_Nd, the largest eigenvalue of H (Alg. 1), by k Lanczos steps (oracle; test infrastructure only).

Alg. 1 takes lam_Nd, the largest eigenvalue of H, as the upper end of the interval
the Chebyshev filter damps, and leaves open how it is found.  Reading used here (the
standard one for Chebyshev-filtered subspace iteration, Zhou and Li's bound
estimator): from a normalised start vector v_1, k Lanczos steps

    w = H v_j - beta_{j-1} v_{j-1},   alpha_j = v_j^T w,
    w = w - alpha_j v_j,              beta_j = ||w||,   v_{j+1} = w / beta_j

give the tridiagonal T_k = tridiag(beta, alpha, beta).  Its largest eigenvalue
theta_k is a Ritz value of H, hence never above lam_Nd, and approaches it quickly
because the top of a discretised Laplacian's spectrum is dense and well separated
from the start vector's bulk.  With s the eigenvector of T_k for theta_k, the Ritz
pair's residual is ||H y - theta_k y|| = |beta_k s_k| (beta_k = norm of the last
Lanczos residual vector), so an eigenvalue of H lies within that distance of
theta_k; theta_k + |beta_k s_k| is returned as the estimate of lam_Nd (once the
largest Ritz value has converged it is an upper bound).  No reorthogonalisation:
lost orthogonality only duplicates converged Ritz values, it does not move the
largest one.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import apply_h


def lanczos_coefficients(prob, v0, k):
    """(alpha[0:k], beta[0:k]) of k Lanczos steps on H from v0 (stops early if beta hits 0)."""
    v = np.array(v0, dtype=np.float64).reshape(-1)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for _ in range(k):
        w = apply_h(prob, v[:, None])[:, 0] - beta * v_prev
        alpha = float(v @ w)
        w = w - alpha * v
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        if beta == 0.0:
            break
        v_prev, v = v, w / beta
    return np.array(alphas), np.array(betas)


def tridiagonal_max(alphas, betas):
    """Largest eigenvalue of the symmetric tridiagonal matrix with diagonal alphas and
    off-diagonal betas[:-1], and the last component of its unit eigenvector."""
    k = len(alphas)
    w, s = scipy.linalg.eigh_tridiagonal(alphas, betas[:k - 1], select="i", select_range=(k - 1, k - 1))
    return float(w[0]), float(s[-1, 0])


def lanczos_upper_bound(prob, v0, k):
    """(theta_k + |beta_k s_k|, theta_k, |beta_k s_k|, alphas, betas) for k Lanczos steps from v0."""
    a, b = lanczos_coefficients(prob, v0, k)
    theta, s_last = tridiagonal_max(a, b)
    resid = abs(b[-1] * s_last)
    return theta + resid, theta, resid, a, b
