"""Pins of the complex (Bloch wavevector) oracle against facts it does not compute itself:
the real oracle at k = 0, the FD symbol on Bloch plane waves, Hermiticity, the supercell
folding of the spectrum, and convergence of the complex CheFSI step to the lowest
eigenvalues of the dense H_k."""
import numpy as np
import pytest

from oracle import hamiltonian as oh
from oracle import kpoint as ok
from oracle.fd import second_derivative_weights
from paper_2302_09708_amd import inputs


def _problem(n, h, atoms, fd_order=6, veff=None, nproj=4):
    bc = (0, 0, 0)
    atoms = np.asarray(atoms, dtype=float)
    if veff is None:
        veff = inputs.gaussian_wells(n, h, bc, atoms)
    sp, si, npj, chi, gam = inputs.kb_projectors(n, h, bc, atoms, nproj)
    return inputs.Problem(tuple(n), tuple(h), bc, fd_order, veff, atoms, sp, si, npj, chi, gam)


N, H = (8, 7, 7), (0.55, 0.5, 0.55)          # L = 4.4 x 3.5 x 3.85 bohr, above 2 rc = 3
ATOMS = [[0.25, 1.1, 3.6], [2.6, 2.9, 1.7]]   # the first one's support wraps in x and z


def test_k0_is_the_real_hamiltonian():
    prob = _problem(N, H, ATOMS)
    img = inputs.support_images(prob)
    x = np.random.default_rng(0).standard_normal((prob.nd, 3))
    assert np.abs(ok.apply_h_k(prob, img, (0.0, 0.0, 0.0), x) - oh.apply_h(prob, x)).max() < 1e-12


@pytest.mark.parametrize("k,m", [((0.3, -0.2, 0.5), (1, 0, -2)), ((1.1, 0.7, -0.4), (0, 3, 1))])
def test_bloch_plane_waves_have_the_fd_symbol(k, m):
    """exp(i (k + G).r), G_d = 2 pi m_d / L_d: T_k psi = eps psi with
    eps = -1/2 sum_d h_d^-2 (w_0 + 2 sum_p w_p cos((k_d + G_d) p h_d))."""
    prob = _problem((9, 8, 7), (0.4, 0.45, 0.5), np.zeros((0, 3)), fd_order=8,
                    veff=np.zeros(9 * 8 * 7), nproj=1)
    w = second_derivative_weights(prob.fd_order)
    L = [prob.n[d] * prob.h[d] for d in range(3)]
    q = [k[d] + 2 * np.pi * m[d] / L[d] for d in range(3)]
    z, y, x = np.meshgrid(*(np.arange(prob.n[d]) * prob.h[d] for d in (2, 1, 0)), indexing="ij")
    psi = np.exp(1j * (q[0] * x + q[1] * y + q[2] * z)).reshape(-1)
    eps = -0.5 * sum((w[0] + 2 * sum(w[p] * np.cos(q[d] * p * prob.h[d]) for p in range(1, len(w))))
                     / prob.h[d] ** 2 for d in range(3))
    t = ok.kinetic_k(prob, psi[:, None], k)[:, 0]
    assert np.abs(t - eps * psi).max() < 1e-10 * abs(eps)


def test_dense_h_k_is_hermitian_and_depends_on_k():
    prob = _problem(N, H, ATOMS)
    img = inputs.support_images(prob)
    assert np.abs(img).max() == 1  # some supports wrap
    hk = ok.dense_h_k(prob, img, (0.4, -0.3, 0.2))
    assert np.abs(hk - hk.conj().T).max() < 1e-12
    h0 = ok.dense_h_k(prob, img, (0.0, 0.0, 0.0))
    assert np.abs(hk - h0).max() > 1e-3


def test_supercell_folds_three_wavevectors():
    """The cell tripled along x (atoms repeated, Veff tiled) at k = 0 has exactly the union
    of the cell's spectra at k_x = 0, 2 pi / (3 L_x) and 4 pi / (3 L_x).  With a phase of
    exp(2 pi i / 3) a projector phase of the wrong sign (or none) breaks the union; the
    plane-wave test fixes the kinetic sign."""
    cell = _problem(N, H, ATOMS)
    lx = N[0] * H[0]
    n3 = (3 * N[0], N[1], N[2])
    v3 = np.tile(cell.veff.reshape(N[2], N[1], N[0]), (1, 1, 3)).reshape(-1)
    atoms3 = np.vstack([np.asarray(ATOMS) + [j * lx, 0.0, 0.0] for j in range(3)])
    sup = _problem(n3, H, atoms3, veff=v3)
    ev_sup = np.linalg.eigvalsh(oh.dense_h(sup))
    img = inputs.support_images(cell)
    evs = [np.linalg.eigvalsh(ok.dense_h_k(cell, img, (2 * np.pi * j / (3 * lx), 0.0, 0.0))) for j in range(3)]
    assert np.abs(np.sort(np.concatenate(evs)) - ev_sup).max() < 1e-9 * np.abs(ev_sup).max()
    # not the same as folding k = 0 three times (the phase matters)
    assert np.abs(np.sort(np.concatenate([evs[0]] * 3)) - ev_sup).max() > 1e-3


def test_complex_step_converges_to_lowest_eigenvalues():
    prob = _problem(N, H, ATOMS)
    img = inputs.support_images(prob)
    k = (0.5, 0.2, -0.3)
    ev = np.linalg.eigvalsh(ok.dense_h_k(prob, img, k))
    ns = 12
    rng = np.random.default_rng(3)
    x = rng.standard_normal((prob.nd, ns)) + 1j * rng.standard_normal((prob.nd, ns))
    lo, cut, hi = ev[0] - 0.5, ev[0] + 0.1 * (ev[-1] - ev[0]), ev[-1] + 0.1
    for _ in range(14):
        d, x = ok.chefsi_step_k(prob, img, k, x, 10, lo, cut, hi)
        lo, cut = d[0], d[-1]
    assert np.abs(d[:8] - ev[:8]).max() < 1e-8
    assert np.abs(x.conj().T @ x - np.eye(ns)).max() < 1e-10  # Ms-orthonormal rotation
