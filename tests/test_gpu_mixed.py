"""Parity of the mixed-precision path (FP32 filter, split-bf16 MFMA projection and
rotation, FP64 dense stage and FP64 refinement) with the FP64 CPU oracle.

Kernel tolerances come from the arithmetic.  With hi = bf16(x), lo = bf16(x - hi)
(round to nearest, 8 significant bits) every FP32 value is x = hi + lo + e with
|e| <= 2^-16 |x|, and the three kept products miss at most 3.1 * 2^-16 |a b| of a b.
Products of bf16 values are exact in FP32; summing K of them in FP32 adds at most
K * 2^-24 sum |a b|.  So for every output element

    |C - C_exact| <= (3.1 * 2^-16 + K * 2^-24) * sum_k |a_k b_k|  (+ 2^-24 |C| when stored as FP32)

with K the number of terms summed in FP32 (the K chunk of the projection, Ns for
the rotation).  Whole iterations are held to the stated mixed-precision bar after
the FP64 refinement: Ritz values within 1e-5 Ha of the FP64 oracle and a subspace
residual of at most 1e-5.
"""
import numpy as np
import pytest

from oracle import chefsi as oc
from paper_2302_09708_amd import inputs
from tests._gpu import dev, dev_square, host, host_square

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U16 = 2.0 ** -16
U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


def _handle(cs, prob, ns, precision):
    h = cs.Handle(prob, precision=precision, max_ns=ns)
    return h, cs.workspace(h, ns)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ns >= 768 runs the 256-wide tile kernel: 800 (7 tiles of 128, the last 256-wide tile half
# used) and 1031 (9 tiles of 128, a ragged last tile)
@pytest.mark.parametrize("shape,ns", [((30, 31, 29), 137), ((9, 7, 6), 3), ((16, 16, 16), 128), ((30, 31, 29), 800),
                                      ((28, 27, 26), 1031)])
def test_project_split_bf16(cs, shape, ns):
    """Hs = X^T H X and Ms = X^T X from an FP32 block: split-bf16 bound, element by element."""
    from oracle.hamiltonian import apply_h
    prob = inputs.small_problem(n=shape, bc=(0, 1, 0), n_atoms=4, nproj_per_atom=4, seed=6)
    X = _f32(np.random.default_rng(5).standard_normal((prob.nd, ns)))
    h, ws = _handle(cs, prob, ns, cs.MIXED)
    Hs = torch.zeros(ns, ns, dtype=torch.float64, device="cuda")
    Ms = torch.zeros_like(Hs)
    h.chefsi_project(dev(X, "float32"), ns, Hs, Ms, ws)
    # the FP32 product H X the kernel contracts with, from the FP32 apply
    Y = torch.zeros(ns, prob.nd, dtype=torch.float32, device="cuda")
    h.chefsi_apply_h(dev(X, "float32"), Y, ns, ws)
    torch.cuda.synchronize()
    hs, ms = host_square(Hs), host_square(Ms)
    y = host(Y)
    assert np.array_equal(hs, hs.T) and np.array_equal(ms, ms.T)
    y_ref = apply_h(prob, X)
    assert np.abs(y - y_ref).max() <= 2e-6 * max(abs(v) for v in oc.spectral_bounds(prob)) * np.abs(X).max()
    kchunk = prob.nd  # an upper bound on the FP32-summed K chunk
    rel = 3.1 * U16 + kchunk * U24
    up = np.triu(np.ones((ns, ns), dtype=bool))  # the kernel forms the upper triangle and mirrors it
    ms_ex, hs_ex = X.T @ X, X.T @ y
    assert np.all((np.abs(ms - ms_ex) <= rel * (np.abs(X).T @ np.abs(X)))[up])
    assert np.all((np.abs(hs - hs_ex) <= rel * (np.abs(X).T @ np.abs(y)))[up])
    # and far inside the worst case for random data
    assert np.abs(ms - ms_ex).max() <= 1e-5 * np.abs(ms_ex).max()
    assert np.abs(hs - hs_ex)[up].max() <= 1e-5 * np.abs(hs_ex).max()


@pytest.mark.parametrize("ns", [1, 16, 137, 300])
def test_rotate_split_bf16(cs, ns):
    prob = inputs.small_problem(n=(21, 20, 19), n_atoms=0, nproj_per_atom=0, seed=1)
    rng = np.random.default_rng(ns)
    X = _f32(rng.standard_normal((prob.nd, ns)))
    Z = rng.standard_normal((ns, ns))
    h, ws = _handle(cs, prob, ns, cs.MIXED)
    Xd = dev(X, "float32")
    h.chefsi_rotate(Xd, dev_square(Z), ns, ws)
    torch.cuda.synchronize()
    ref = X @ Z
    got = host(Xd)
    bound = (3.1 * U16 + ns * U24) * (np.abs(X) @ np.abs(Z)) + U24 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()


def _run_oracle(name):
    cfg = inputs.CONFIGS[name]
    prob = inputs.make_problem(cfg)
    X0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed).T
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, x_ref = oc.chefsi(prob, X0, cfg.degree, cfg.n_iter, lo, cut, hi)
    return cfg, prob, X0, (lo, cut, hi), d_ref, x_ref


@pytest.fixture(scope="module")
def cfg1_ref():
    return _run_oracle("cfg1")


@pytest.fixture(scope="module")
def slab_ref():
    return _run_oracle("slab_small")


def _check_mixed_solve(cs, ref, label):
    cfg, prob, X0, bounds, d_ref, x_ref = ref
    h, ws = _handle(cs, prob, cfg.ns, cs.MIXED)
    Xd = dev(X0, "float32")
    d, lo, cut = h.solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, ws, bounds=bounds)
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    x = host(Xd)
    err = np.abs(d[:k] - d_ref[:k]).max()
    rho = oc.subspace_residual(x_ref, x, k)
    print(f"{label} mixed: N_chk={k} max|dRitz|={err:.3e} Ha subspace residual={rho:.3e}", flush=True)
    assert err <= 1e-5
    assert rho <= 1e-5
    assert np.abs(x.T @ x - np.eye(cfg.ns)).max() <= 1e-5
    assert np.all(np.diff(d) >= 0)


def test_solve_mixed_cfg1_refined(cs, cfg1_ref):
    _check_mixed_solve(cs, cfg1_ref, "cfg1")


def test_solve_mixed_slab_refined(cs, slab_ref):
    _check_mixed_solve(cs, slab_ref, "slab 16x16x48 (Dirichlet z)")


def test_solve_fp64_slab(cs, slab_ref):
    cfg, prob, X0, (lo, cut, hi), d_ref, x_ref = slab_ref
    h, ws = _handle(cs, prob, cfg.ns, cs.FP64)
    Xd = dev(X0)
    d, _, _ = h.chefsi_solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, lo, cut, hi, ws)
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    assert np.abs(d - d_ref).max() <= 1e-10
    assert oc.subspace_residual(x_ref, host(Xd), k) <= 1e-8


def test_mixed_step_ritz_and_determinism(cs, cfg1_ref):
    """One unrefined mixed step: Ritz values near the FP64 step's, bitwise repeatable."""
    cfg, prob, X0, (lo, cut, hi), _, _ = cfg1_ref
    d_ref, _ = oc.chefsi_step(prob, X0, cfg.degree, lo, cut, hi)
    h, ws = _handle(cs, prob, cfg.ns, cs.MIXED)
    outs = []
    for _ in range(2):
        Xd = dev(X0, "float32")
        d = h.chefsi_step(Xd, cfg.ns, cfg.degree, lo, cut, hi, ws)
        outs.append((d, host(Xd)))
    print("cfg1 one mixed step: max|dRitz| =", np.abs(outs[0][0] - d_ref).max(), flush=True)
    assert np.abs(outs[0][0] - d_ref).max() <= 1e-3
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("n", [(14, 13, 12), (26, 25, 27)])
def test_refine_degree0_is_fp64_rayleigh_ritz(cs, n):
    """degree 0: Rayleigh-Ritz of the stored block with FP64 arithmetic (no filter).  The
    FP32 block goes through FP64 row panels: 2184 points are four whole panels, 17550
    points are four panels of two K chunks and a last panel of six rows."""
    prob = inputs.small_problem(n=n, n_atoms=3, nproj_per_atom=4, seed=3)
    ns = 24
    X = _f32(np.random.default_rng(2).standard_normal((prob.nd, ns)))
    hs, ms = oc.project(prob, X)
    d_ref, z_ref = oc.diagonalize(hs, ms)
    for prec, dt in ((cs.MIXED, "float32"), (cs.FP64, "float64")):
        h, ws = _handle(cs, prob, ns, prec)
        Xd = dev(X, dt)
        d = h.chefsi_refine_fp64(Xd, ns, ws, 0)
        assert np.abs(d - d_ref).max() <= 1e-10 * np.abs(d_ref).max()
        x = host(Xd)
        ref = X @ z_ref
        x = x * np.sign(np.sum(x * ref, axis=0))[None, :]  # eigenvectors up to sign
        tol = 1e-6 if prec == cs.MIXED else 1e-11
        assert np.abs(x - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("prec_name", ["mixed", "fp64"])
def test_projection_and_eigh_with_widely_scaled_columns(cs, prec_name):
    """Column norms from 1e-4 to 1e4 (cond(Ms) ~ 1e16): the diagonally scaled Cholesky still
    factors the pencil, and the Ritz values do not depend on the column scaling."""
    prec = cs.MIXED if prec_name == "mixed" else cs.FP64
    dt = "float32" if prec == cs.MIXED else "float64"
    prob = inputs.small_problem(n=(14, 13, 12), n_atoms=3, nproj_per_atom=4, seed=3)
    ns = 48
    rng = np.random.default_rng(4)
    base = rng.standard_normal((prob.nd, ns))
    scale = 10.0 ** np.linspace(-4, 4, ns)
    X = base * scale[None, :]
    if prec == cs.MIXED:
        X = _f32(X)
    hs, ms = oc.project(prob, X / scale[None, :])  # same subspace, unit-scale columns
    d_ref, _ = oc.diagonalize(hs, ms)
    h, ws = _handle(cs, prob, ns, prec)
    Hs = torch.zeros(ns, ns, dtype=torch.float64, device="cuda")
    Ms = torch.zeros_like(Hs)
    h.chefsi_project(dev(X, dt), ns, Hs, Ms, ws)
    D = torch.zeros(ns, dtype=torch.float64, device="cuda")
    h.chefsi_eigh(Hs, Ms, D, ns, ws)
    d = D.cpu().numpy()
    tol = 2e-4 if prec == cs.MIXED else 1e-8
    print(f"{prec_name}: max |dRitz| / max |Ritz| = {np.abs(d - d_ref).max() / np.abs(d_ref).max():.2e}", flush=True)
    assert np.abs(d - d_ref).max() <= tol * np.abs(d_ref).max()


@pytest.mark.parametrize("k", [241, 93])
def test_mixed_falls_back_to_fp64_on_ill_conditioned_blocks(cs, k):
    """Small grids carrying many orbitals and deep wells (serving requests 241: Cholesky of the
    split-bf16 overlap fails; 93: its Ritz values overshoot the spectral bound): the mixed path
    redoes those steps in FP64 and ends within the mixed bar of the FP64 path."""
    prob, ns, degree, seed = inputs.serving_request(k)
    x0 = inputs.initial_block(prob.nd, ns, seed)
    out = {}
    for prec, dt in ((cs.FP64, "float64"), (cs.MIXED, "float32")):
        h, ws = _handle(cs, prob, ns, prec)
        h.chefsi_profile_reset()
        Xd = torch.from_numpy(x0).to(device="cuda", dtype=getattr(torch, dt))
        d, _, _ = h.solve(Xd, ns, degree, 10, ws)
        out[prec] = (d, h.chefsi_profile_read(cs.PROF_FALLBACK)[1])
    d64, dmx = out[cs.FP64][0], out[cs.MIXED][0]
    kchk = oc.gap_index(d64, int(ns / 1.2))
    err = np.abs(dmx[:kchk] - d64[:kchk]).max()
    print(f"request {k}: N={prob.n[0]} ns={ns} fallback steps={out[cs.MIXED][1]} N_chk={kchk} "
          f"max|dRitz| vs FP64 = {err:.2e}", flush=True)
    assert out[cs.MIXED][1] >= 1
    assert err <= 1e-5


def _golden_twin(name="cfg3_twin_ritz.txt"):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    rows, bounds = [], None
    for line in open(path):
        if line.startswith("# bounds of the first step"):
            bounds = tuple(float(v) for v in line.split(":")[1].split())
        elif not line.startswith("#") and line.strip():
            rows.append(np.array([float(v) for v in line.split()]))
    return bounds, rows


def test_cfg3_twin_solves_against_stored_oracle_ritz_values(cs):
    """The reduced slab workload (30 x 30 x 90, Dirichlet z, 25 atoms, Ns 300, degree 24,
    6 filter passes): FP64 solve against the oracle's Ritz values (stored by
    tests/golden/make_cfg3_twin_ritz.py, which runs only the oracle: its 6 iterations take
    ~15 minutes on the host) to 1e-10 Ha; mixed solve (5 mixed steps + FP64 refinement) to
    1e-5 Ha on the gap-bounded leading block.  The mixed subspace is compared with the FP64
    solve's (rho <= 1e-5), whose subspace the oracle pins on the smaller workloads and whose
    Ritz values it pins here; the mixed block's residuals are checked with the oracle's H."""
    from oracle.hamiltonian import apply_h
    cfg = inputs.CONFIGS["cfg3_twin"]
    prob = inputs.make_problem(cfg)
    bounds, rows = _golden_twin()
    d_ref = rows[cfg.n_iter - 1]
    lo, cut, hi = oc.spectral_bounds(prob)
    assert np.allclose((lo, cut, hi), bounds, rtol=1e-14, atol=0)
    x0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed)
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    out = {}
    for prec, dt in ((cs.FP64, "float64"), (cs.MIXED, "float32")):
        h, ws = _handle(cs, prob, cfg.ns, prec)
        Xd = torch.from_numpy(x0).to(device="cuda", dtype=getattr(torch, dt))
        d, _, _ = h.solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, ws, bounds=(lo, cut, hi))
        out[prec] = (d, host(Xd))
        h.close()
    d64, x64 = out[cs.FP64]
    dmx, xmx = out[cs.MIXED]
    err64 = np.abs(d64 - d_ref).max()
    errmx = np.abs(dmx[:k] - d_ref[:k]).max()
    rho = oc.subspace_residual(x64, xmx, k)
    res = oc.residual_norms(prob, xmx[:, :k], dmx[:k])
    res64 = oc.residual_norms(prob, x64[:, :k], d64[:k])
    print(f"cfg3 twin: N_chk={k} FP64 max|dRitz|={err64:.2e} mixed max|dRitz|={errmx:.2e} rho(mixed, FP64)={rho:.2e} "
          f"max residual mixed {res.max():.2e} FP64 {res64.max():.2e}", flush=True)
    assert err64 <= 1e-10
    assert errmx <= 1e-5
    assert rho <= 1e-5
    assert np.abs(xmx.T @ xmx - np.eye(cfg.ns)).max() <= 1e-5
    assert res.max() <= res64.max() + 1e-4 * max(abs(lo), abs(hi))


def test_cfg4_twin_solves_against_stored_oracle_ritz_values(cs):
    """The reduced cfg4 workload (60^3 periodic at h = 0.22, 125 atoms x 4 projectors from a
    jittered FCC 4^3 lattice: cfg4's spacing and atom density; Ns 900, degree 16, 6 filter
    passes): FP64 solve against the oracle's Ritz values (stored by
    tests/golden/make_cfg4_twin_ritz.py, oracle only, ~80 minutes on the host) to 1e-10 Ha;
    mixed solve (5 mixed steps + FP64 refinement) to 1e-5 Ha on the gap-bounded leading
    block, its subspace against the FP64 solve's (rho <= 1e-5), and the residuals of every
    tenth leading mixed vector under the oracle's H against the FP64 solve's."""
    cfg = inputs.CONFIGS["cfg4_twin"]
    prob = inputs.make_problem(cfg)
    bounds, rows = _golden_twin("cfg4_twin_ritz.txt")
    assert len(rows) == cfg.n_iter
    d_ref = rows[cfg.n_iter - 1]
    lo, cut, hi = oc.spectral_bounds(prob)
    assert np.allclose((lo, cut, hi), bounds, rtol=1e-14, atol=0)
    x0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed)
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    out = {}
    for prec, dt in ((cs.FP64, "float64"), (cs.MIXED, "float32")):
        print(f"cfg4 twin solve precision {prec}", flush=True)
        h, ws = _handle(cs, prob, cfg.ns, prec)
        Xd = torch.from_numpy(x0).to(device="cuda", dtype=getattr(torch, dt))
        d, _, _ = h.solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, ws, bounds=(lo, cut, hi))
        out[prec] = (d, host(Xd))
        h.close()
        del Xd, ws
        torch.cuda.empty_cache()
    d64, x64 = out[cs.FP64]
    dmx, xmx = out[cs.MIXED]
    err64 = np.abs(d64 - d_ref).max()
    errmx = np.abs(dmx[:k] - d_ref[:k]).max()
    rho = oc.subspace_residual(x64, xmx, k)
    cols = np.arange(0, k, 10)
    res = oc.residual_norms(prob, xmx[:, cols], dmx[cols])
    res64 = oc.residual_norms(prob, x64[:, cols], d64[cols])
    print(f"cfg4 twin: N_chk={k} FP64 max|dRitz|={err64:.2e} mixed max|dRitz|={errmx:.2e} rho(mixed, FP64)={rho:.2e} "
          f"max residual mixed {res.max():.2e} FP64 {res64.max():.2e}", flush=True)
    assert err64 <= 1e-10
    assert errmx <= 1e-5
    assert rho <= 1e-5
    assert np.abs(xmx.T @ xmx - np.eye(cfg.ns)).max() <= 1e-5
    assert res.max() <= res64.max() + 1e-4 * max(abs(lo), abs(hi))


def test_cfg2_ten_iterations_against_stored_oracle_ritz_values(cs):
    """The headline workload itself (72^3 periodic at h = 0.25, 128 atoms x 4 projectors,
    Ns 600, degree 20, 10 filter passes from the seeded X0): FP64 solve against the oracle's
    Ritz values after 10 iterations (stored by tests/golden/make_cfg2_ritz.py, oracle only,
    ~35 minutes on the host) to 1e-10 Ha on all Ns; mixed solve (9 mixed steps + FP64
    refinement) to 1e-5 Ha on the gap-bounded leading block, its subspace against the FP64
    solve's (rho <= 1e-5), and the residuals of every twentieth leading vector under the
    oracle's H."""
    cfg = inputs.CONFIGS["cfg2"]
    prob = inputs.make_problem(cfg)
    bounds, rows = _golden_twin("cfg2_ritz.txt")
    assert len(rows) == cfg.n_iter
    d_ref = rows[cfg.n_iter - 1]
    lo, cut, hi = oc.spectral_bounds(prob)
    assert np.allclose((lo, cut, hi), bounds, rtol=1e-14, atol=0)
    x0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed)
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    out = {}
    for prec, dt in ((cs.FP64, "float64"), (cs.MIXED, "float32")):
        print(f"cfg2 solve precision {prec}", flush=True)
        h, ws = _handle(cs, prob, cfg.ns, prec)
        Xd = torch.from_numpy(x0).to(device="cuda", dtype=getattr(torch, dt))
        d, _, _ = h.solve(Xd, cfg.ns, cfg.degree, cfg.n_iter, ws, bounds=(lo, cut, hi))
        out[prec] = (d, host(Xd))
        h.close()
        del Xd, ws
        torch.cuda.empty_cache()
    d64, x64 = out[cs.FP64]
    dmx, xmx = out[cs.MIXED]
    err64 = np.abs(d64 - d_ref).max()
    errmx = np.abs(dmx[:k] - d_ref[:k]).max()
    rho = oc.subspace_residual(x64, xmx, k)
    cols = np.arange(0, k, 20)
    res = oc.residual_norms(prob, xmx[:, cols], dmx[cols])
    res64 = oc.residual_norms(prob, x64[:, cols], d64[cols])
    print(f"cfg2: N_chk={k} FP64 max|dRitz|={err64:.2e} mixed max|dRitz|={errmx:.2e} rho(mixed, FP64)={rho:.2e} "
          f"max residual mixed {res.max():.2e} FP64 {res64.max():.2e}", flush=True)
    assert err64 <= 1e-10
    assert errmx <= 1e-5
    assert rho <= 1e-5
    assert np.abs(xmx.T @ xmx - np.eye(cfg.ns)).max() <= 1e-5
    assert res.max() <= res64.max() + 1e-4 * max(abs(lo), abs(hi))
