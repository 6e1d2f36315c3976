"""Planted mistakes in the oracle must fail at least one pin (CPU only).

Each case swaps one oracle function for a copy with a single plausible error
(dropped term, wrong sign, wrong index, transposed operand) and checks that a
pin from the other test modules then fails.
"""
import numpy as np
import pytest

import oracle.chefsi as oc
import oracle.hamiltonian as oh
import oracle.kpoint as ok
from oracle.fd import second_derivative_weights
from tests import test_oracle_chefsi as tc
from tests import test_oracle_hamiltonian as th
from tests import test_oracle_kpoint as tk


def _kinetic_wrong_index(prob, x):
    nx, ny, nz = prob.n
    w = second_derivative_weights(prob.fd_order)
    r = len(w) - 1
    u = x.reshape(nz, ny, nx, x.shape[1])
    lap = np.zeros_like(u)
    for d in range(3):
        inv_h2 = 1.0 / prob.h[d] ** 2
        lap += w[0] * inv_h2 * u
        for p in range(1, r + 1):
            q = p + 1 if p < r else p          # planted: shifts by the wrong distance
            lap += w[p] * inv_h2 * (oh._shift(u, q, d, prob.bc[d] == 0) + oh._shift(u, -q, d, prob.bc[d] == 0))
    return (-0.5 * lap).reshape(-1, x.shape[1])


def _kinetic_dirichlet_as_periodic(prob, x):
    class P:  # planted: boundary conditions ignored
        pass
    p = P()
    p.n, p.h, p.fd_order, p.bc = prob.n, prob.h, prob.fd_order, (0, 0, 0)
    return _orig_kinetic(p, x)


def _local_wrong_sign(prob, x):
    return -prob.veff[:, None] * x


def _nonlocal_no_dv(prob, x):
    y = np.zeros_like(x)
    for idx, chi, gam in oh.atom_blocks(prob):
        y[idx, :] += chi @ (gam[:, None] * (chi.T @ x[idx, :]))
    return y


def _atom_blocks_transposed(prob):
    coff = goff = 0
    for J in range(len(prob.nproj)):
        lo, hi = int(prob.supp_ptr[J]), int(prob.supp_ptr[J + 1])
        nj, npj = hi - lo, int(prob.nproj[J])
        chi = np.asarray(prob.chi[coff:coff + nj * npj]).reshape(nj, npj)   # planted: row-major read
        yield np.asarray(prob.supp_idx[lo:hi], np.int64), chi, np.asarray(prob.gamma[goff:goff + npj])
        coff += nj * npj
        goff += npj


def _filter_dropped_term(prob, x, degree, lam_lo, lam_cut, lam_hi):
    c, e = 0.5 * (lam_hi + lam_cut), 0.5 * (lam_hi - lam_cut)
    s1 = e / (lam_lo - c)
    s, y_prev = s1, np.array(x)
    y = (s1 / e) * (oh.apply_h(prob, y_prev) - c * y_prev)
    for _ in range(1, degree):
        s_next = 1.0 / (2.0 / s1 - s)
        y_prev, y = y, (2.0 * s_next / e) * (oh.apply_h(prob, y) - c * y)   # planted: no Y_{k-1} term
        s = s_next
    return y


def _diag_swapped_operands(hs, ms):
    import scipy.linalg
    return scipy.linalg.eigh(ms, hs + 1e3 * np.eye(len(hs)), type=1)    # planted: H and M swapped


_orig_kinetic = oh.kinetic

CASES = [
    ("kinetic", _kinetic_wrong_index, lambda: th.test_periodic_free_particle_full_spectrum(
        (6, 5, 7), (0.3, 0.35, 0.4), 4)),
    ("kinetic", _kinetic_dirichlet_as_periodic, lambda: th.test_separable_potential_matches_1d_sums(
        (0, 1, 1), 6)),
    ("local_potential", _local_wrong_sign, lambda: th.test_separable_potential_matches_1d_sums(
        (0, 1, 1), 6)),
    ("nonlocal_potential", _nonlocal_no_dv, th.test_rank_one_constant_projector_moves_zero_mode_to_gamma),
    ("atom_blocks", _atom_blocks_transposed, th.test_plane_wave_projectors_rank_four),
]


@pytest.mark.parametrize("name,mutant,pin", CASES, ids=[c[1].__name__ for c in CASES])
def test_hamiltonian_mutant_is_caught(monkeypatch, name, mutant, pin):
    monkeypatch.setattr(oh, name, mutant)
    with pytest.raises(AssertionError):
        pin()


def test_filter_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(oc, "chebyshev_filter", _filter_dropped_term)
    with pytest.raises(AssertionError):
        tc.test_filter_plane_wave_gains()


def test_diagonalize_mutant_is_caught(monkeypatch):
    monkeypatch.setattr(oc, "diagonalize", _diag_swapped_operands)
    with pytest.raises(AssertionError):
        tc.test_diagonalize_agrees_with_independent_routes()


# ---- the complex (Bloch wavevector) oracle -------------------------------------------
_orig_blocks_k = ok.projector_blocks_k
_orig_bloch_shift = ok._bloch_shift


def _projector_phase_conjugated(prob, img, k):
    for idx, chi, gam in _orig_blocks_k(prob, img, k):
        yield idx, chi.conj(), gam                  # planted: exp(-i k.mL) instead of exp(+i k.mL)


def _projector_phase_dropped(prob, img, k):
    for idx, chi, gam in _orig_blocks_k(prob, img, k):
        yield idx, chi.real.astype(complex), gam    # planted: no Bloch phase on the projectors


def _ghost_phase_conjugated(u, p, d, periodic, phase):
    return _orig_bloch_shift(u, p, d, periodic, np.conj(phase))   # planted: wrong sign of k in the ghosts


def _project_k_no_conjugate(prob, img, k, xf):
    yf = ok.apply_h_k(prob, img, k, xf)
    hs = xf.T @ yf                                  # planted: transpose without conjugation
    ms = xf.conj().T @ xf
    return 0.5 * (hs + hs.conj().T), 0.5 * (ms + ms.conj().T)


KCASES = [
    ("projector_blocks_k", _projector_phase_conjugated, tk.test_supercell_folds_three_wavevectors),
    ("projector_blocks_k", _projector_phase_dropped, tk.test_supercell_folds_three_wavevectors),
    ("_bloch_shift", _ghost_phase_conjugated,
     lambda: tk.test_bloch_plane_waves_have_the_fd_symbol((0.3, -0.2, 0.5), (1, 0, -2))),
    ("project_k", _project_k_no_conjugate, tk.test_complex_step_converges_to_lowest_eigenvalues),
]


@pytest.mark.parametrize("name,mutant,pin", KCASES, ids=[c[1].__name__ for c in KCASES])
def test_kpoint_mutant_is_caught(monkeypatch, name, mutant, pin):
    monkeypatch.setattr(ok, name, mutant)
    with pytest.raises(AssertionError):
        pin()
