"""The seeded synthetic inputs: determinism, layout and the stated recipe."""
import numpy as np
import pytest

from paper_2302_09708_amd import inputs


def test_cfg1_recipe_and_determinism():
    cfg = inputs.CONFIGS["cfg1"]
    a = inputs.make_problem(cfg)
    b = inputs.make_problem(cfg)
    assert a.nd == 24 ** 3 and a.n_atoms == 8
    np.testing.assert_array_equal(a.veff, b.veff)
    np.testing.assert_array_equal(a.chi, b.chi)
    assert -2.0 * 8 <= a.veff.min() < -1.0 and a.veff.max() <= 0.0
    x = inputs.initial_block(a.nd, cfg.ns, cfg.x_seed)
    assert x.shape == (40, a.nd)
    np.testing.assert_array_equal(x, inputs.initial_block(a.nd, cfg.ns, cfg.x_seed))


@pytest.mark.parametrize("bc,npa", [((0, 0, 0), 1), ((0, 0, 1), 4), ((1, 1, 1), 4)])
def test_projector_layout_and_normalisation(bc, npa):
    p = inputs.small_problem(n=(12, 11, 13), bc=bc, n_atoms=4, nproj_per_atom=npa, seed=3)
    assert p.supp_ptr[0] == 0 and p.supp_ptr[-1] == len(p.supp_idx)
    coff = 0
    for J in range(p.n_atoms):
        idx = p.supp_idx[p.supp_ptr[J]:p.supp_ptr[J + 1]]
        assert np.all(np.diff(idx) > 0)                      # sorted, unique
        assert idx.min() >= 0 and idx.max() < p.nd
        nj, npj = len(idx), int(p.nproj[J])
        chi = p.chi[coff:coff + nj * npj].reshape(npj, nj)   # column-major n_J x np_J
        np.testing.assert_allclose((chi * chi).sum(axis=1) * p.dv, 1.0, rtol=1e-12)
        coff += nj * npj
    assert coff == len(p.chi) and len(p.gamma) == int(p.nproj.sum())


def test_support_radius_cfg2_shape():
    cfg = inputs.CONFIGS["cfg2"]
    atoms = inputs.atom_positions(cfg)
    assert atoms.shape == (128, 3)
    sp, si, npj, chi, gam = inputs.kb_projectors(cfg.n, cfg.h, cfg.bc, atoms[:2], 4)
    # a sphere of radius 1.5 bohr at h = 0.25 holds ~ 4/3 pi 6^3 = 905 points
    assert 850 < sp[1] - sp[0] < 960


def test_serving_requests_are_in_range():
    for k in range(20):
        prob, ns, deg, seed = inputs.serving_request(k)
        N = prob.n[0]
        assert 24 <= N <= 64 and 8 <= prob.n_atoms <= 96
        assert 1 <= ns <= min(400, N ** 3 // 8) and deg == 20
        assert prob.bc in ((0, 0, 0), (0, 0, 1))
