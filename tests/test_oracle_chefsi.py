"""Pins for the oracle's CheFSI step (Algorithm 1: filtering, projection, diagonalisation, rotation)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import chefsi as oc
from oracle.fd import second_derivative_weights
from oracle.hamiltonian import apply_h, dense_h
from paper_2302_09708_amd.inputs import initial_block, small_problem
from tests.test_oracle_hamiltonian import bare_problem, free_particle_energies


def _cos_modes(n, ks):
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return np.stack([np.cos(2 * np.pi * (kx * x / n[0] + ky * y / n[1] + kz * z / n[2])).reshape(-1)
                     for (kx, ky, kz) in ks], axis=1)


def test_filter_plane_wave_gains():
    """V = 0, periodic: a cosine mode of energy E leaves the filter multiplied by T_m(L(E)) / T_m(L(lam_lo))."""
    n, h, order, m = (24, 24, 24), (0.3, 0.3, 0.3), 12, 20
    prob = bare_problem(n, h, (0, 0, 0), order)
    ks = [(0, 0, 0), (1, 0, 0), (2, 1, 0), (3, 3, 3), (12, 0, 5), (12, 12, 12)]
    e = free_particle_energies(n, h, order).reshape(n[2], n[1], n[0])
    E = np.array([e[kz, ky, kx] for (kx, ky, kz) in ks])
    X = _cos_modes(n, ks)
    lam_lo, lam_cut, lam_hi = -0.3, 1.0, float(e.max()) + 0.5
    c, ee = 0.5 * (lam_hi + lam_cut), 0.5 * (lam_hi - lam_cut)
    gain = np.array([oc.chebyshev_t(m, (x - c) / ee) for x in E])
    scale = oc.chebyshev_t(m, (lam_lo - c) / ee)
    Yu = oc.chebyshev_filter_unscaled(prob, X, m, lam_cut, lam_hi)
    np.testing.assert_allclose(Yu, X * gain[None, :], rtol=0, atol=1e-9 * np.abs(gain).max())
    Ys = oc.chebyshev_filter(prob, X, m, lam_lo, lam_cut, lam_hi)
    np.testing.assert_allclose(Ys, X * (gain / scale)[None, :], rtol=0, atol=1e-12)


def test_scaled_filter_is_unscaled_divided_by_scalar():
    prob = small_problem(n=(10, 9, 11), bc=(0, 0, 1), n_atoms=2, nproj_per_atom=4, seed=2)
    X = np.random.default_rng(4).standard_normal((prob.nd, 6))
    lo, cut, hi = oc.spectral_bounds(prob)
    for m in (1, 2, 7, 16):
        c, e = 0.5 * (hi + cut), 0.5 * (hi - cut)
        ys = oc.chebyshev_filter(prob, X, m, lo, cut, hi)
        yu = oc.chebyshev_filter_unscaled(prob, X, m, cut, hi)
        np.testing.assert_allclose(ys * oc.chebyshev_t(m, (lo - c) / e), yu,
                                   rtol=1e-11, atol=1e-11 * np.abs(yu).max())


def test_filter_scalars_are_ratios_of_chebyshev_values():
    m, lo, cut, hi = 16, -2.3, 4.0, 130.0
    c, e, ss = oc.filter_scalars(m, lo, cut, hi)
    l0 = (lo - c) / e
    for k in range(1, m + 1):
        assert abs(ss[k - 1] - oc.chebyshev_t(k - 1, l0) / oc.chebyshev_t(k, l0)) < 1e-13


def test_diagonalize_agrees_with_independent_routes():
    rng = np.random.default_rng(7)
    k = 37
    a = rng.standard_normal((200, k)) @ np.diag(np.logspace(0, 2, k))
    ms = a.T @ a
    b = rng.standard_normal((k, k))
    hs = b + b.T
    d, z = oc.diagonalize(hs, ms)
    assert np.all(np.diff(d) >= 0)
    np.testing.assert_allclose(z.T @ ms @ z, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(hs @ z - ms @ z * d[None, :], 0, atol=1e-9 * np.abs(hs).max())
    d2, z2 = oc.diagonalize_by_cholesky(hs, ms)
    np.testing.assert_allclose(d2, d, atol=1e-10 * np.abs(d).max())
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(ms, hs)).real)
    np.testing.assert_allclose(ev, d, atol=1e-8 * np.abs(d).max())


def test_step_invariants_and_rayleigh_ritz_bounds():
    prob = small_problem(n=(9, 10, 8), bc=(0, 1, 0), n_atoms=3, nproj_per_atom=4, seed=8)
    lam = np.linalg.eigvalsh(dense_h(prob))
    X0 = initial_block(prob.nd, 14, 99).T
    lo, cut, hi = oc.spectral_bounds(prob)
    assert lo <= lam[0] and hi >= lam[-1]
    d, X = oc.chefsi_step(prob, X0, 10, lo, cut, hi)
    np.testing.assert_allclose(X.T @ X, np.eye(14), atol=1e-10)   # Z^T M Z = I  =>  X^T X = I
    assert np.all(np.diff(d) >= 0)
    assert np.all(d >= lam[:14] - 1e-10)                           # Courant-Fischer: Ritz >= exact
    # the Ritz values are the eigenvalues of X^T H X for the rotated block
    np.testing.assert_allclose(np.diag(X.T @ apply_h(prob, X)), d, atol=1e-10)


def test_chefsi_converges_to_dense_spectrum():
    prob = small_problem(n=(10, 9, 12), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), n_atoms=3, nproj_per_atom=4, seed=12)
    lam = np.linalg.eigvalsh(dense_h(prob))
    ns = 24
    X0 = initial_block(prob.nd, ns, 5).T
    lo, cut, hi = oc.spectral_bounds(prob)
    d, X = oc.chefsi(prob, X0, 14, 25, lo, cut, hi)
    k = oc.gap_index(d, 18)
    assert k >= 12
    np.testing.assert_allclose(d[:k], lam[:k], atol=1e-9)
    assert oc.residual_norms(prob, X[:, :k], d[:k]).max() < 1e-6


def test_chefsi_free_particle_shells_on_cfg1_grid():
    """cfg1 grid (24^3, h = 0.3, order 12), V = 0: converged Ritz values are the closed-form shells
    0, 0.3808 (x6), 0.7615 (x12), 1.1423 (x8), 1.5231 (x6)."""
    n, h, order = (24, 24, 24), (0.3, 0.3, 0.3), 12
    prob = bare_problem(n, h, (0, 0, 0), order)
    ref = np.sort(free_particle_energies(n, h, order))
    assert abs(ref[1] - 0.380772) < 1e-6 and abs(ref[32] - 1.523087) < 1e-6
    X0 = initial_block(prob.nd, 40, 2001).T
    lo, cut, hi = oc.spectral_bounds(prob)
    d, X = oc.chefsi(prob, X0, 20, 14, lo, cut, hi)
    np.testing.assert_allclose(d[:33], ref[:33], atol=1e-9)


def test_spectral_bounds_are_tight_for_free_particles():
    n, h, order = (8, 6, 10), (0.3, 0.35, 0.25), 12
    prob = bare_problem(n, h, (0, 0, 0), order)
    lo, cut, hi = oc.spectral_bounds(prob)
    ref = free_particle_energies(n, h, order)
    assert abs(hi - ref.max()) < 1e-10 * ref.max()       # Gershgorin = symbol at theta = pi (even N)
    assert lo == 0.0 and abs(cut - 0.1 * hi) < 1e-12


def test_spectral_bounds_enclose_spectrum_with_projectors():
    for seed, bc in [(1, (0, 0, 0)), (2, (0, 0, 1)), (3, (1, 1, 1))]:
        prob = small_problem(n=(9, 8, 10), bc=bc, n_atoms=3, nproj_per_atom=4, seed=seed)
        lam = np.linalg.eigvalsh(dense_h(prob))
        lo, cut, hi = oc.spectral_bounds(prob)
        assert lo <= lam[0] + 1e-12 and hi >= lam[-1] - 1e-12


def test_metrics():
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((50, 6)))
    assert oc.subspace_residual(q, q @ scipy.linalg.qr(rng.standard_normal((6, 6)))[0], 6) < 1e-12
    assert abs(oc.subspace_residual(q[:, :3], q[:, 3:], 3) - 1.0) < 1e-12
    assert oc.gap_index(np.array([0.0, 1.0, 1.0, 1.0005, 2.0]), 4) == 4
    assert oc.gap_index(np.array([0.0, 1.0, 1.0, 1.0005, 2.0]), 3) == 1
