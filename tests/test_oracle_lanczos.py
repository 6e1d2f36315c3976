"""Pins for the oracle's Lanczos estimate of lam_Nd (the largest eigenvalue of H in Alg. 1).

Expected values come from other routes: the Fourier closed form of the periodic
FD Laplacian, dense eigensolves of tiny Hamiltonians, the tridiagonal form of H
in an orthonormal Krylov basis built by QR, and the rigorous Gershgorin bound.
"""
import numpy as np
import pytest

from oracle.chefsi import spectral_bounds
from oracle.hamiltonian import apply_h, dense_h
from oracle.lanczos import lanczos_coefficients, lanczos_upper_bound, tridiagonal_max
from paper_2302_09708_amd.inputs import CONFIGS, initial_block, make_problem, small_problem
from tests.test_oracle_hamiltonian import bare_problem, free_particle_energies


def test_free_particle_cfg1_grid_closed_form():
    n, h, order = (24, 24, 24), (0.3, 0.3, 0.3), 12
    prob = bare_problem(n, h, (0, 0, 0), order)
    lam_max = float(free_particle_energies(n, h, order).max())
    v0 = initial_block(prob.nd, 1, 2001)[0]
    bound, theta, resid, _, _ = lanczos_upper_bound(prob, v0, 40)
    assert theta <= lam_max * (1 + 1e-12)          # a Ritz value never exceeds lam_Nd
    assert theta >= lam_max * (1 - 1e-5)           # and has converged close to it
    assert theta <= lam_max <= bound + 1e-12 * lam_max   # the residual interval covers lam_Nd
    bound10, theta10, _, _, _ = lanczos_upper_bound(prob, v0, 10)
    assert theta10 < theta and bound10 - theta10 > bound - theta   # fewer steps: lower, wider


@pytest.mark.parametrize("bc,na", [((0, 0, 0), 3), ((0, 0, 1), 2), ((1, 1, 1), 0)])
def test_tiny_hamiltonian_against_dense(bc, na):
    prob = small_problem(n=(7, 6, 8), h=(0.3, 0.28, 0.33), bc=bc, fd_order=12, n_atoms=na,
                         nproj_per_atom=4 if na else 0, seed=21)
    H = dense_h(prob)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    v0 = np.random.default_rng(3).standard_normal(prob.nd)
    bound, theta, _, _, _ = lanczos_upper_bound(prob, v0, 30)
    assert theta <= ev[-1] + 1e-10 * abs(ev[-1])
    assert bound >= ev[-1] - 1e-10 * abs(ev[-1])
    # a Krylov space of full dimension reproduces the top of the spectrum
    _, theta_full, _, _, _ = lanczos_upper_bound(prob, v0, prob.nd)
    assert abs(theta_full - ev[-1]) <= 1e-9 * abs(ev[-1])


def test_coefficients_are_h_in_a_qr_krylov_basis():
    prob = small_problem(n=(9, 8, 7), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), fd_order=8, n_atoms=2, seed=4)
    v0 = np.random.default_rng(7).standard_normal(prob.nd)
    k = 6
    a, b = lanczos_coefficients(prob, v0, k)
    K = np.empty((prob.nd, k))
    K[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(1, k):
        K[:, j] = apply_h(prob, K[:, j - 1:j])[:, 0]
    Q, R = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(R))[None, :]           # same orientation as the Lanczos vectors
    T = Q.T @ apply_h(prob, Q)
    np.testing.assert_allclose(a, np.diag(T), rtol=0, atol=1e-9 * np.abs(a).max())
    np.testing.assert_allclose(b[:k - 1], np.diag(T, 1), rtol=0, atol=1e-9 * np.abs(a).max())
    assert tridiagonal_max(a, b)[0] == pytest.approx(np.linalg.eigvalsh(0.5 * (T + T.T))[-1], rel=1e-12)


def test_below_the_gershgorin_bound_on_cfg1():
    prob = make_problem(CONFIGS["cfg1"])
    lam_hi = spectral_bounds(prob)[2]
    v0 = initial_block(prob.nd, 1, 2001)[0]
    bound, theta, _, _, _ = lanczos_upper_bound(prob, v0, 30)
    assert theta < bound <= lam_hi
