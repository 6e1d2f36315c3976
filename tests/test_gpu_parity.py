"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Tolerances (FP64 path): kernels that only reorder a fixed sum are compared at
~1e-13 of the scale of the cancelling terms; whole steps at the stated Ritz
bar of 1e-10 Ha and a subspace residual of 1e-8 (sin of the largest principal
angle against the oracle's subspace, over a Ritz-gap-bounded leading block).
"""
import numpy as np
import pytest

from oracle import chefsi as oc
from oracle.hamiltonian import apply_h
from paper_2302_09708_amd import inputs
from tests._gpu import dev, dev_square, host, host_square, stencil_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


def _handle(cs, prob, ns, precision=0):
    h = cs.Handle(prob, precision=precision, max_ns=ns)
    ws = cs.workspace(h, ns)
    return h, ws


APPLY_CASES = [
    # (n, bc, order, atoms, proj/atom, ns)
    ((37, 29, 23), (0, 0, 0), 12, 3, 4, 9),
    ((24, 24, 24), (0, 0, 0), 12, 8, 1, 5),
    ((20, 33, 17), (0, 1, 1), 8, 2, 4, 6),
    ((6, 7, 6), (0, 0, 0), 12, 1, 4, 3),      # minimal periodic n = r
    ((1, 9, 5), (1, 1, 1), 4, 0, 0, 2),       # a one-point direction
    ((130, 12, 9), (0, 1, 0), 6, 2, 4, 4),    # rows wider than two waves
    ((45, 40, 50), (1, 0, 1), 2, 4, 4, 7),
    ((64, 64, 64), (0, 0, 1), 12, 6, 4, 3),
    ((16, 15, 14), (0, 0, 0), 12, 12, 4, 5),  # up to 8 atoms' supports on one point (32 entries)
]


@pytest.mark.parametrize("case", APPLY_CASES, ids=[str(c[0]) + str(c[1]) + f"o{c[2]}" for c in APPLY_CASES])
def test_apply_h_fp64(cs, case):
    n, bc, order, na, npa, ns = case
    print(f"apply_h fp64 {case}", flush=True)
    prob = inputs.small_problem(n=n, h=(0.3, 0.27, 0.33), bc=bc, fd_order=order, n_atoms=na,
                                nproj_per_atom=npa, seed=sum(n))
    X = np.random.default_rng(1).standard_normal((prob.nd, ns))
    ref = apply_h(prob, X)
    h, ws = _handle(cs, prob, ns)
    Xd, Yd = dev(X), torch.zeros(ns, prob.nd, dtype=torch.float64, device="cuda")
    h.chefsi_apply_h(Xd, Yd, ns, ws)
    torch.cuda.synchronize()
    got = host(Yd)
    scale = stencil_scale(prob) * np.abs(X).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale * 10


FP32_CASES = APPLY_CASES[:4] + APPLY_CASES[-1:]


@pytest.mark.parametrize("case", FP32_CASES, ids=[str(c[0]) for c in FP32_CASES])
def test_apply_h_fp32_mixed_handle(cs, case):
    n, bc, order, na, npa, ns = case
    prob = inputs.small_problem(n=n, h=(0.3, 0.27, 0.33), bc=bc, fd_order=order, n_atoms=na,
                                nproj_per_atom=npa, seed=sum(n))
    X = np.random.default_rng(2).standard_normal((prob.nd, ns)).astype(np.float32)
    ref = apply_h(prob, X.astype(np.float64))
    h, ws = _handle(cs, prob, ns, precision=cs.MIXED)
    Xd, Yd = dev(X, "float32"), torch.zeros(ns, prob.nd, dtype=torch.float32, device="cuda")
    h.chefsi_apply_h(Xd, Yd, ns, ws)
    torch.cuda.synchronize()
    scale = stencil_scale(prob) * np.abs(X).max()
    assert np.abs(host(Yd) - ref).max() <= 2e-6 * scale


@pytest.mark.parametrize("degree", [1, 8, 9])
def test_filter_fp64(cs, degree):
    prob = inputs.small_problem(n=(20, 18, 22), bc=(0, 0, 0), n_atoms=3, nproj_per_atom=4, seed=4)
    ns = 7
    X = np.random.default_rng(3).standard_normal((prob.nd, ns))
    lo, cut, hi = oc.spectral_bounds(prob)
    ref = oc.chebyshev_filter(prob, X, degree, lo, cut, hi)
    h, ws = _handle(cs, prob, ns)
    Xd = dev(X)
    h.chefsi_filter(Xd, ns, degree, lo, cut, hi, ws)
    torch.cuda.synchronize()
    assert np.abs(host(Xd) - ref).max() <= 1e-11 * np.abs(ref).max()


def test_project_fp64_ragged_tiles(cs):
    prob = inputs.small_problem(n=(30, 31, 29), bc=(0, 1, 0), n_atoms=4, nproj_per_atom=4, seed=6)
    ns = 137                      # two 128-wide tiles, ragged; Nd = 26970 not a multiple of 16
    X = np.random.default_rng(5).standard_normal((prob.nd, ns))
    hs_ref, ms_ref = oc.project(prob, X)
    h, ws = _handle(cs, prob, ns)
    Hs = torch.zeros(ns, ns, dtype=torch.float64, device="cuda")
    Ms = torch.zeros_like(Hs)
    h.chefsi_project(dev(X), ns, Hs, Ms, ws)
    torch.cuda.synchronize()
    hs, ms = host_square(Hs), host_square(Ms)
    assert np.array_equal(hs, hs.T) and np.array_equal(ms, ms.T)
    assert np.abs(ms - ms_ref).max() <= 1e-13 * np.abs(ms_ref).max()
    assert np.abs(hs - hs_ref).max() <= 1e-12 * np.abs(hs_ref).max()


@pytest.mark.parametrize("ns", [1, 16, 137, 300])
def test_rotate_fp64(cs, ns):
    prob = inputs.small_problem(n=(21, 20, 19), n_atoms=0, nproj_per_atom=0, seed=1)
    rng = np.random.default_rng(ns)
    X = rng.standard_normal((prob.nd, ns))
    Z = rng.standard_normal((ns, ns))
    h, ws = _handle(cs, prob, ns)
    Xd = dev(X)
    h.chefsi_rotate(Xd, dev_square(Z), ns, ws)
    torch.cuda.synchronize()
    ref = X @ Z
    assert np.abs(host(Xd) - ref).max() <= 1e-13 * np.abs(X).max() * np.abs(Z).sum(axis=0).max()


def test_eigh_fp64(cs):
    prob = inputs.small_problem(n=(12, 12, 12), n_atoms=0, nproj_per_atom=0, seed=1)
    ns = 137
    rng = np.random.default_rng(9)
    a = rng.standard_normal((400, ns))
    ms = a.T @ a
    b = rng.standard_normal((ns, ns))
    hs = b + b.T
    h, ws = _handle(cs, prob, ns)
    Hd, Md = dev_square(hs), dev_square(ms)
    D = torch.zeros(ns, dtype=torch.float64, device="cuda")
    h.chefsi_eigh(Hd, Md, D, ns, ws)
    torch.cuda.synchronize()
    d_ref, _ = oc.diagonalize(hs, ms)
    d = D.cpu().numpy()
    z = host_square(Hd)
    assert np.abs(d - d_ref).max() <= 1e-10 * np.abs(d_ref).max()
    assert np.abs(z.T @ ms @ z - np.eye(ns)).max() <= 1e-9
    assert np.abs(hs @ z - ms @ z * d[None, :]).max() <= 1e-9 * np.abs(hs).max()


def _cfg1():
    cfg = inputs.CONFIGS["cfg1"]
    prob = inputs.make_problem(cfg)
    X0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed).T
    return cfg, prob, X0


def test_step_fp64_cfg1(cs):
    cfg, prob, X0 = _cfg1()
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, x_ref = oc.chefsi_step(prob, X0, cfg.degree, lo, cut, hi)
    h, ws = _handle(cs, prob, cfg.ns)
    lo_l, cut_l, hi_l = h.chefsi_spectral_bounds()
    assert abs(lo_l - lo) <= 1e-12 * abs(lo) and abs(hi_l - hi) <= 1e-12 * hi and abs(cut_l - cut) <= 1e-11 * hi
    Xd = dev(X0)
    d = h.chefsi_step(Xd, cfg.ns, cfg.degree, lo, cut, hi, ws)
    assert np.abs(d - d_ref).max() <= 1e-10
    x = host(Xd)
    assert np.abs(x.T @ x - np.eye(cfg.ns)).max() <= 1e-10
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    assert k >= 10
    assert oc.subspace_residual(x_ref, x, k) <= 1e-8


def test_solve_fp64_cfg1_ten_iterations(cs):
    cfg, prob, X0 = _cfg1()
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, x_ref = oc.chefsi(prob, X0, cfg.degree, cfg.n_iter, lo, cut, hi)
    h, ws = _handle(cs, prob, cfg.ns)
    Xd = dev(X0)
    d, lo_out, cut_out = h.chefsi_solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, lo, cut, hi, ws)
    print("cfg1 10 it: max |dRitz| =", np.abs(d - d_ref).max(), flush=True)
    assert np.abs(d - d_ref).max() <= 1e-10
    assert lo_out == d[0] and cut_out == d[-1]
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    assert oc.subspace_residual(x_ref, host(Xd), k) <= 1e-8
    # converged part: residual of the Ritz pairs
    assert oc.residual_norms(prob, host(Xd)[:, :k], d[:k]).max() < 1e-3


def test_step_is_bitwise_deterministic(cs):
    cfg, prob, X0 = _cfg1()
    lo, cut, hi = oc.spectral_bounds(prob)
    h, ws = _handle(cs, prob, cfg.ns)
    outs = []
    for _ in range(2):
        Xd = dev(X0)
        d = h.chefsi_step(Xd, cfg.ns, cfg.degree, lo, cut, hi, ws)
        outs.append((d, host(Xd)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_error_paths_and_handle_reuse(cs):
    cfg, prob, X0 = _cfg1()
    ns = 12
    lo, cut, hi = oc.spectral_bounds(prob)
    h, ws = _handle(cs, prob, ns)
    Xd = dev(X0[:, :ns])
    with pytest.raises(cs.ChefsiError) as e:
        h.chefsi_step(Xd, ns, 4, lo, cut, hi, ws, ws_bytes=h.chefsi_workspace_bytes(ns) - 1)
    assert e.value.status == cs.ERR_WORKSPACE
    with pytest.raises(cs.ChefsiError) as e:
        h.chefsi_step(Xd, ns + 1, 4, lo, cut, hi, ws)
    assert e.value.status == cs.ERR_INVALID_ARG
    with pytest.raises(cs.ChefsiError) as e:
        h.chefsi_step(Xd, ns, 4, hi, cut, lo, ws)
    assert e.value.status == cs.ERR_INVALID_ARG
    # rank-deficient block: a zero column stays exactly zero through the filter, so the
    # overlap matrix has an exactly zero pivot (duplicated columns would leave a pivot
    # at rounding level whose sign is not determined)
    Xdup = X0[:, :ns].copy()
    Xdup[:, 5] = 0.0
    with pytest.raises(cs.ChefsiError) as e:
        h.chefsi_step(dev(Xdup), ns, 4, lo, cut, hi, ws)
    assert e.value.status == cs.ERR_NOT_POSDEF
    assert h.chefsi_last_info() == ns + 6
    # an indefinite overlap matrix given straight to the dense stage
    Hs = dev_square(np.eye(ns))
    Ms = dev_square(np.diag(np.r_[np.ones(ns - 1), -1.0]))
    D = torch.zeros(ns, dtype=torch.float64, device="cuda")
    with pytest.raises(cs.ChefsiError) as e:
        h.chefsi_eigh(Hs, Ms, D, ns, ws)
    assert e.value.status == cs.ERR_NOT_POSDEF
    # the handle still works
    d = h.chefsi_step(Xd, ns, 4, lo, cut, hi, ws)
    d_ref, _ = oc.chefsi_step(prob, X0[:, :ns], 4, lo, cut, hi)
    assert np.abs(d - d_ref).max() <= 1e-10


def test_full_size_cfg2_sampled(cs):
    """cfg2 at full size in the benchmark's launch configuration: H X on sampled columns
    against the oracle, and Rayleigh-Ritz properties of one step on sampled entries."""
    cfg = inputs.CONFIGS["cfg2"]
    prob = inputs.make_problem(cfg)
    ns = cfg.ns
    print("cfg2 full size: building X0", flush=True)
    torch.manual_seed(0)
    X = torch.randn(ns, prob.nd, dtype=torch.float64, device="cuda")
    h, ws = _handle(cs, prob, ns)
    Y = torch.empty_like(X)
    h.chefsi_apply_h(X, Y, ns, ws)
    torch.cuda.synchronize()
    cols = [0, 1, 299, 598, 599]
    xs = X[cols].cpu().numpy().T
    ref = apply_h(prob, xs)
    got = Y[cols].cpu().numpy().T
    scale = stencil_scale(prob) * np.abs(xs).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale
    del Y
    lo, cut, hi = h.chefsi_spectral_bounds()
    print("cfg2 full size: one step", flush=True)
    d = h.chefsi_step(X, ns, cfg.degree, lo, cut, hi, ws)
    assert np.all(np.isfinite(d)) and np.all(np.diff(d) >= 0) and d[0] >= lo - 1e-9
    xs = X[cols].cpu().numpy().T
    assert np.abs(xs.T @ xs - np.eye(len(cols))).max() <= 1e-9        # orthonormal columns
    rq = np.einsum("ij,ij->j", xs, apply_h(prob, xs))                  # Rayleigh quotients = Ritz values
    assert np.abs(rq - d[cols]).max() <= 1e-9 * max(1.0, np.abs(d).max())
