"""Pins for the oracle's matrix-free Hamiltonian (Section 2.1: stencil, Veff, nonlocal projectors).

Every expected value here comes from a route other than the oracle's own
shift-and-add code: Fourier closed forms of the periodic FD Laplacian,
Toeplitz/circulant 1-D matrices for separable problems, the textbook
second-order Dirichlet spectrum, exact rank-one / rank-four updates, and the
secular equation of a rank-one perturbation evaluated through an FFT.
"""
import numpy as np
import pytest

from oracle.fd import second_derivative_weights
from oracle.hamiltonian import apply_h, dense_h, nonlocal_potential
from paper_2302_09708_amd.inputs import Problem, small_problem


def bare_problem(n, h, bc, order, veff=None, atoms=None):
    """A problem with optional potential and an explicit list of atoms [(idx, chi (n_J x np_J), gamma)]."""
    nd = int(np.prod(n))
    veff = np.zeros(nd) if veff is None else np.asarray(veff, dtype=np.float64)
    ptr, idx, npj, chi, gam = [0], [], [], [], []
    for (i, c, g) in (atoms or []):
        i = np.asarray(i, dtype=np.int32)
        c = np.asarray(c, dtype=np.float64).reshape(len(i), -1)
        ptr.append(ptr[-1] + len(i))
        idx.append(i)
        npj.append(c.shape[1])
        chi.append(c.T.reshape(-1))       # column-major n_J x np_J
        gam.append(np.asarray(g, dtype=np.float64).reshape(-1))
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return Problem(tuple(n), tuple(h), tuple(bc), order, veff, np.zeros((len(npj), 3)),
                   np.array(ptr, np.int64), cat(idx, np.int32), np.array(npj, np.int32),
                   cat(chi, np.float64), cat(gam, np.float64))


def free_particle_energies(n, h, order):
    """Closed form of the periodic FD kinetic spectrum: E = 1/2 sum_d s(2 pi k_d / N_d) / h_d^2,
    s(theta) = -w_0 - 2 sum_p w_p cos(p theta); one value per Fourier mode (k_x, k_y, k_z)."""
    w = second_derivative_weights(order)
    per_dim = []
    for d in range(3):
        th = 2 * np.pi * np.arange(n[d]) / n[d]
        s = -w[0] - 2 * sum(w[p] * np.cos(p * th) for p in range(1, len(w)))
        per_dim.append(0.5 * s / h[d] ** 2)
    e = per_dim[2][:, None, None] + per_dim[1][None, :, None] + per_dim[0][None, None, :]
    return e.reshape(-1)  # index order matches (kz, ky, kx)


def one_dim_matrix(N, h, order, periodic, v=None):
    """-1/2 d^2/dx^2 (FD) + diag(v) as a dense N x N matrix: circulant (periodic) or truncated Toeplitz."""
    w = second_derivative_weights(order)
    r = len(w) - 1
    a = np.zeros((N, N))
    for i in range(N):
        for p in range(-r, r + 1):
            j = i + p
            if periodic:
                a[i, j % N] += w[abs(p)]
            elif 0 <= j < N:
                a[i, j] += w[abs(p)]
    a *= -0.5 / (h * h)
    if v is not None:
        a += np.diag(v)
    return a


@pytest.mark.parametrize("n,h,order", [
    ((6, 5, 7), (0.3, 0.35, 0.4), 4),
    ((4, 5, 6), (0.3, 0.3, 0.3), 12),     # N < 2r: stencil wraps more than once
    ((9, 8, 10), (0.25, 0.3, 0.35), 12),
    ((7, 7, 7), (0.3, 0.3, 0.3), 8),
])
def test_periodic_free_particle_full_spectrum(n, h, order):
    H = dense_h(bare_problem(n, h, (0, 0, 0), order))
    got = np.linalg.eigvalsh(0.5 * (H + H.T))
    ref = np.sort(free_particle_energies(n, h, order))
    np.testing.assert_allclose(got, ref, atol=1e-10 * ref.max())


def test_plane_waves_are_eigenvectors_cfg1_grid():
    n, h, order = (24, 24, 24), (0.3, 0.3, 0.3), 12
    prob = bare_problem(n, h, (0, 0, 0), order)
    e = free_particle_energies(n, h, order).reshape(n[2], n[1], n[0])
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    cols, ens = [], []
    for (kx, ky, kz) in [(0, 0, 0), (1, 0, 0), (1, 2, 3), (12, 12, 12), (5, 11, 7), (23, 1, 0)]:
        ph = 2 * np.pi * (kx * x / n[0] + ky * y / n[1] + kz * z / n[2])
        cols.append(np.cos(ph).reshape(-1))
        ens.append(e[kz, ky, kx])
    X = np.stack(cols, axis=1)
    np.testing.assert_allclose(apply_h(prob, X), X * np.array(ens)[None, :], atol=1e-10)


@pytest.mark.parametrize("bc,order", [((0, 1, 1), 6), ((1, 1, 1), 12), ((1, 0, 0), 12)])
def test_separable_potential_matches_1d_sums(bc, order):
    n, h = (7, 6, 8), (0.3, 0.25, 0.35)
    rng = np.random.default_rng(11)
    v1 = [rng.uniform(-2.0, 1.0, size=n[d]) for d in range(3)]
    veff = (v1[2][:, None, None] + v1[1][None, :, None] + v1[0][None, None, :]).reshape(-1)
    H = dense_h(bare_problem(n, h, bc, order, veff=veff))
    got = np.linalg.eigvalsh(0.5 * (H + H.T))
    e1 = [np.linalg.eigvalsh(one_dim_matrix(n[d], h[d], order, bc[d] == 0, v1[d])) for d in range(3)]
    ref = np.sort((e1[2][:, None, None] + e1[1][None, :, None] + e1[0][None, None, :]).reshape(-1))
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


def test_second_order_dirichlet_closed_form():
    n, h = (5, 6, 7), (0.3, 0.4, 0.5)
    for d in range(3):  # the 1-D construction itself against the textbook spectrum
        j = np.arange(1, n[d] + 1)
        ref1 = 0.5 * (4.0 / h[d] ** 2) * np.sin(j * np.pi / (2 * (n[d] + 1))) ** 2
        np.testing.assert_allclose(np.linalg.eigvalsh(one_dim_matrix(n[d], h[d], 2, False)), np.sort(ref1),
                                   rtol=1e-13)
    H = dense_h(bare_problem(n, h, (1, 1, 1), 2))
    e1 = [0.5 * (4.0 / h[d] ** 2) * np.sin(np.arange(1, n[d] + 1) * np.pi / (2 * (n[d] + 1))) ** 2
          for d in range(3)]
    ref = np.sort((e1[2][:, None, None] + e1[1][None, :, None] + e1[0][None, None, :]).reshape(-1))
    np.testing.assert_allclose(np.linalg.eigvalsh(H), ref, atol=1e-11 * ref.max())


def test_rank_one_constant_projector_moves_zero_mode_to_gamma():
    n, h, order, gamma = (6, 6, 6), (0.3, 0.3, 0.3), 6, 0.7
    nd, dv = 216, 0.027
    chi = np.full((nd, 1), 1.0 / np.sqrt(nd * dv))      # sum chi^2 dV = 1
    prob = bare_problem(n, h, (0, 0, 0), order, atoms=[(np.arange(nd), chi, [gamma])])
    got = np.linalg.eigvalsh(dense_h(prob))
    ref = free_particle_energies(n, h, order)
    ref = np.sort(np.concatenate([ref[ref > 1e-12], [gamma]]))
    np.testing.assert_allclose(got, ref, atol=1e-11)


def test_plane_wave_projectors_rank_four():
    """Four orthonormal cosine modes as the projectors of one atom: each mode's energy moves by its gamma."""
    n, h, order = (8, 6, 10), (0.3, 0.35, 0.25), 12
    nd, dv = int(np.prod(n)), 0.3 * 0.35 * 0.25
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    ks = [(1, 0, 0), (0, 2, 1), (3, 1, 2), (1, 1, 4)]
    gam = np.array([0.3, 0.5, 0.7, 1.1])
    e = free_particle_energies(n, h, order).reshape(n[2], n[1], n[0])
    chi = np.zeros((nd, 4))
    for a, (kx, ky, kz) in enumerate(ks):
        c = np.cos(2 * np.pi * (kx * x / n[0] + ky * y / n[1] + kz * z / n[2])).reshape(-1)
        chi[:, a] = c / np.sqrt((c * c).sum() * dv)
    prob = bare_problem(n, h, (0, 0, 0), order, atoms=[(np.arange(nd), chi, gam)])
    got = np.linalg.eigvalsh(0.5 * (dense_h(prob) + dense_h(prob).T))
    ref = list(free_particle_energies(n, h, order))
    for a, (kx, ky, kz) in enumerate(ks):
        ea = e[kz, ky, kx]
        j = int(np.argmin(np.abs(np.array(ref) - ea)))
        ref[j] = ea + gam[a]
    np.testing.assert_allclose(got, np.sort(ref), atol=1e-10)


def _secular_spectrum(n, h, order, v_unit, gamma):
    """Eigenvalues of T + gamma v v^T (periodic T, ||v|| = 1) from the secular equation
    1 + gamma sum_k |<phi_k, v>|^2 / (E_k - lam) = 0, with Fourier weights from an FFT."""
    e = free_particle_energies(n, h, order).reshape(n[2], n[1], n[0])
    wts = np.abs(np.fft.fftn(v_unit.reshape(n[2], n[1], n[0]))) ** 2 / v_unit.size
    e, wts = e.reshape(-1), wts.reshape(-1)
    order_idx = np.argsort(e)
    e, wts = e[order_idx], wts[order_idx]
    # group degenerate energies
    levels, weights, mult = [], [], []
    for ek, wk in zip(e, wts):
        if levels and abs(ek - levels[-1]) <= 1e-11 * max(1.0, abs(ek)):
            weights[-1] += wk
            mult[-1] += 1
        else:
            levels.append(ek)
            weights.append(wk)
            mult.append(1)
    levels, weights = np.array(levels), np.array(weights)
    poles = levels[weights > 1e-26]
    pw = weights[weights > 1e-26]
    f = lambda lam: 1.0 + gamma * np.sum(pw / (poles - lam))
    roots = []
    uppers = list(poles[1:]) + [poles[-1] + gamma * pw.sum() + 1.0]
    for lo, hi in zip(poles, uppers):
        a, b = lo, hi
        for _ in range(200):
            mid = 0.5 * (a + b)
            if mid == a or mid == b:
                break
            if f(mid) < 0:
                a = mid
            else:
                b = mid
        roots.append(0.5 * (a + b))
    rest = []
    for lv, wv, m in zip(levels, weights, mult):
        rest += [lv] * (m - 1 if wv > 1e-26 else m)
    return np.sort(np.array(roots + rest))


def test_gaussian_projector_secular_equation():
    n, h, order, gamma = (8, 9, 10), (0.3, 0.3, 0.3), 12, 0.5
    prob0 = small_problem(n=n, h=h, bc=(0, 0, 0), fd_order=order, n_atoms=1, nproj_per_atom=1,
                          seed=3, with_veff=False, gamma=gamma)
    nd, dv = prob0.nd, prob0.dv
    v = np.zeros(nd)
    v[prob0.supp_idx] = prob0.chi * np.sqrt(dv)          # unit vector (sum chi^2 dV = 1)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    got = np.linalg.eigvalsh(dense_h(prob0))
    ref = _secular_spectrum(n, h, order, v, gamma)
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_full_hamiltonian_is_symmetric_and_nonlocal_psd():
    prob = small_problem(n=(9, 8, 10), bc=(0, 1, 0), n_atoms=3, nproj_per_atom=4, seed=5)
    H = dense_h(prob)
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    vnl = nonlocal_potential(prob, np.eye(prob.nd))
    assert np.linalg.eigvalsh(0.5 * (vnl + vnl.T)).min() > -1e-12
    assert np.abs(vnl).max() > 0.0


def test_columns_are_independent():
    """Applying H to a block equals applying it column by column."""
    prob = small_problem(n=(10, 9, 8), bc=(0, 0, 1), n_atoms=2, nproj_per_atom=4, seed=9)
    X = np.random.default_rng(1).standard_normal((prob.nd, 5))
    Y = apply_h(prob, X)
    for j in range(5):
        np.testing.assert_allclose(Y[:, j], apply_h(prob, X[:, j]), rtol=0, atol=1e-12)
