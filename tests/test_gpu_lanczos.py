"""Parity of the device Lanczos estimate of lam_Nd (Alg. 1's largest eigenvalue of H)
with the oracle's, through the C-ABI.

FP64 handles: the first coefficients agree with the oracle's to rounding and the
largest Ritz value theta to 1e-10 relative (theta is a converged, well-conditioned
quantity; later coefficients drift apart at the rounding level as orthogonality is
lost the same way but not in the same bits).  Mixed handles store the Lanczos
vectors in FP32: theta agrees to 1e-5 relative.
"""
import time

import numpy as np
import pytest

from oracle import chefsi as oc
from oracle.lanczos import lanczos_upper_bound
from paper_2302_09708_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


def _run(cs, prob, precision, v0, steps):
    h = cs.Handle(prob, precision=precision, max_ns=1)
    ws = torch.empty(h.chefsi_lanczos_workspace_bytes(), dtype=torch.uint8, device="cuda")
    dt = torch.float64 if precision == cs.FP64 else torch.float32
    v = torch.from_numpy(v0).to(device="cuda", dtype=dt)
    out = h.chefsi_lanczos_bound(v, steps, ws)
    assert np.array_equal(v.cpu().numpy(), v0.astype(v.cpu().numpy().dtype))  # v0 untouched
    h.close()
    return out


CASES = [
    ("cfg1", None),
    ("slab", dict(n=(23, 21, 30), h=(0.3, 0.3, 0.3), bc=(0, 0, 1), n_atoms=5, nproj_per_atom=4, seed=8)),
    ("dirichlet", dict(n=(17, 19, 15), h=(0.28, 0.3, 0.33), bc=(1, 1, 1), n_atoms=3, nproj_per_atom=4, seed=9)),
]


def _problem(case):
    name, kw = case
    return inputs.make_problem(inputs.CONFIGS["cfg1"]) if kw is None else inputs.small_problem(**kw)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp64_matches_oracle(cs, case):
    prob = _problem(case)
    print(f"lanczos fp64 {case[0]} nd={prob.nd}", flush=True)
    v0 = inputs.initial_block(prob.nd, 1, 2001)[0]
    steps = 30
    lam, theta, a, b = _run(cs, prob, cs.FP64, v0, steps)
    lam_ref, theta_ref, resid_ref, a_ref, b_ref = lanczos_upper_bound(prob, v0, steps)
    scale = np.abs(a_ref).max()
    np.testing.assert_allclose(a[:8], a_ref[:8], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(b[:8], b_ref[:8], rtol=0, atol=1e-12 * scale)
    assert abs(theta - theta_ref) <= 1e-10 * abs(theta_ref)
    assert lam >= theta and abs(lam - lam_ref) <= 1e-9 * abs(theta_ref) + 0.05 * resid_ref
    assert lam <= oc.spectral_bounds(prob)[2]


def test_mixed_handle_fp32_vectors(cs):
    prob = _problem(CASES[1])
    v0 = inputs.initial_block(prob.nd, 1, 2001)[0]
    lam, theta, a, b = _run(cs, prob, cs.MIXED, v0, 30)
    _, theta_ref, _, _, _ = lanczos_upper_bound(prob, v0, 30)
    assert abs(theta - theta_ref) <= 1e-5 * abs(theta_ref)
    assert lam >= theta


def test_bitwise_reproducible_and_errors(cs):
    prob = _problem(CASES[2])
    v0 = inputs.initial_block(prob.nd, 1, 2001)[0]
    r1 = _run(cs, prob, cs.FP64, v0, 12)
    r2 = _run(cs, prob, cs.FP64, v0, 12)
    assert r1[0] == r2[0] and np.array_equal(r1[2], r2[2]) and np.array_equal(r1[3], r2[3])
    h = cs.Handle(prob, precision=cs.FP64, max_ns=1)
    ws = torch.empty(h.chefsi_lanczos_workspace_bytes(), dtype=torch.uint8, device="cuda")
    v = torch.from_numpy(v0).cuda()
    with pytest.raises(cs.ChefsiError):
        h.chefsi_lanczos_bound(v, 0, ws)
    with pytest.raises(cs.ChefsiError):
        h.chefsi_lanczos_bound(v, 5, ws, ws_bytes=64)
    with pytest.raises(cs.ChefsiError):
        h.chefsi_lanczos_bound(torch.zeros_like(v), 5, ws)
    lam, theta, _, _ = h.chefsi_lanczos_bound(v, 5, ws)  # the handle still works after errors
    assert np.isfinite(lam) and lam >= theta
    h.close()


def test_full_size_cfg2(cs):
    prob = inputs.make_problem(inputs.CONFIGS["cfg2"])
    print("lanczos cfg2 full size", flush=True)
    v0 = inputs.initial_block(prob.nd, 1, 2002)[0]
    steps = 20
    h = cs.Handle(prob, precision=cs.FP64, max_ns=1)
    ws = torch.empty(h.chefsi_lanczos_workspace_bytes(), dtype=torch.uint8, device="cuda")
    v = torch.from_numpy(v0).cuda()
    h.chefsi_lanczos_bound(v, steps, ws)
    t0 = time.perf_counter()
    lam, theta, a, b = h.chefsi_lanczos_bound(v, steps, ws)
    dt = time.perf_counter() - t0
    h.close()
    _, theta_ref, resid_ref, a_ref, _ = lanczos_upper_bound(prob, v0, steps)
    print(f"cfg2: {steps} Lanczos steps {dt * 1e3:.1f} ms, theta {theta:.6f}, lam_Nd {lam:.6f}, "
          f"Gershgorin {oc.spectral_bounds(prob)[2]:.6f}", flush=True)
    assert abs(theta - theta_ref) <= 1e-10 * abs(theta_ref)
    np.testing.assert_allclose(a[:5], a_ref[:5], rtol=0, atol=1e-12 * np.abs(a_ref).max())
