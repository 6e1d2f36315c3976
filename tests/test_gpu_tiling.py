"""Every stencil-pass tiling against the FP64 oracle (Sec. 2.1 stencil + Veff + projectors).

The planner picks rows per thread (PY) and halo values per thread (KH) from the grid
shape; the largest workloads run variants (two rows per thread, four halo values) that
small default grids never select, and autotune also times three and four rows per thread,
which the untuned planner never picks.  chefsi_set_stencil_tiling forces each variant on a
grid small enough for the oracle, for both element types, for H X alone, for the
refinement's FP64 product of an FP32 block, and for a whole mixed solve.  The variants
agree with each other to rounding (the compiler contracts multiply-adds differently per
variant, so the last bits may differ).
"""
import numpy as np
import pytest

from oracle import chefsi as oc
from oracle.hamiltonian import apply_h
from paper_2302_09708_amd import inputs
from tests._gpu import dev, host, stencil_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (rows per thread, row groups): with nx = 40 and r = 6 these give KH = 4, 3 and 2 staged
# values per thread for both PY = 1 and PY = 2, and KH = 4 and 3 for PY = 3, 4 for PY = 4
# (the staged set of a tile of ty rows is 2r (nx + 2r) halo-row values plus 2r ty periodic
# x copies, spread over the block's lanes)
TILINGS = [(1, 4), (1, 8), (1, 24), (2, 4), (2, 6), (2, 12), (3, 4), (3, 8), (4, 6)]
GRIDS = [((40, 24, 16), (0, 0, 0)), ((40, 23, 18), (0, 1, 1))]


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


@pytest.mark.parametrize("grid", GRIDS, ids=[f"{g[0]}{g[1]}" for g in GRIDS])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_h_every_tiling(cs, grid, prec):
    n, bc = grid
    prob = inputs.small_problem(n=n, h=(0.3, 0.27, 0.33), bc=bc, fd_order=12, n_atoms=6, nproj_per_atom=4,
                                seed=sum(n))
    ns = 5
    dt = "float64" if prec == "fp64" else "float32"
    X = np.random.default_rng(7).standard_normal((prob.nd, ns)).astype(dt)
    ref = apply_h(prob, X.astype(np.float64))
    scale = stencil_scale(prob) * np.abs(X).max()
    tol = 1e-12 * scale if prec == "fp64" else 2e-6 * scale
    h = cs.Handle(prob, precision=cs.FP64 if prec == "fp64" else cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    default = h.chefsi_get_stencil_tiling()
    seen, outs = set(), []
    for py, nyg in TILINGS:
        try:
            h.chefsi_set_stencil_tiling(py, nyg)
        except cs.ChefsiError as e:
            assert e.status == cs.ERR_INVALID_ARG
            continue
        t = h.chefsi_get_stencil_tiling()
        assert t[0] == py and t[1] == nyg and t[2] == py * nyg
        print(f"{prec} {n}{bc}: tiling PY={t[0]} groups={t[1]} rows={t[2]} KH={t[3]}", flush=True)
        Yd = torch.zeros(ns, prob.nd, dtype=getattr(torch, dt), device="cuda")
        h.chefsi_apply_h(dev(X, dt), Yd, ns, ws)
        torch.cuda.synchronize()
        got = host(Yd)
        assert np.abs(got - ref).max() <= tol
        seen.add((t[0], t[3]))
        outs.append(got)
    assert {(1, 2), (1, 3), (1, 4), (2, 2), (2, 3), (2, 4), (3, 3), (3, 4), (4, 4)} <= seen
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= (1e-13 if prec == "fp64" else 1e-6) * scale
    h.chefsi_set_stencil_tiling(0, 0)
    assert h.chefsi_get_stencil_tiling() == default


@pytest.mark.parametrize("tiling", [(1, 4), (1, 8), (2, 4), (2, 12)])
def test_refine_degree0_every_tiling(cs, tiling):
    """The refinement's H X in FP64 from an FP32 block (the <float, double, double> pass)."""
    prob = inputs.small_problem(n=(40, 24, 16), bc=(0, 0, 1), n_atoms=5, nproj_per_atom=4, seed=13)
    ns = 12
    X = np.random.default_rng(2).standard_normal((prob.nd, ns)).astype(np.float32).astype(np.float64)
    hs, ms = oc.project(prob, X)
    d_ref, _ = oc.diagonalize(hs, ms)
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    h.chefsi_set_stencil_tiling(*tiling)
    d = h.chefsi_refine_fp64(dev(X, "float32"), ns, ws, 0)
    assert np.abs(d - d_ref).max() <= 1e-10 * np.abs(d_ref).max()


def test_mixed_solve_with_two_rows_and_four_halo_values(cs):
    """A whole mixed solve (mixed steps + FP64 refinement) in the tiling the 120^3 FP32
    workload runs (two rows per thread, four staged values per thread) against the oracle."""
    prob = inputs.small_problem(n=(40, 24, 16), bc=(0, 0, 1), n_atoms=5, nproj_per_atom=4, seed=13)
    ns, degree, n_iter = 24, 12, 5
    x0 = inputs.initial_block(prob.nd, ns, 77).T
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, x_ref = oc.chefsi(prob, x0, degree, n_iter, lo, cut, hi)
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    h.chefsi_set_stencil_tiling(2, 4)
    assert h.chefsi_get_stencil_tiling()[3] == 4
    Xd = dev(x0, "float32")
    d, _, _ = h.solve(Xd, ns, degree, n_iter, ws, bounds=(lo, cut, hi))
    k = oc.gap_index(d_ref, int(ns / 1.2))
    err = np.abs(d[:k] - d_ref[:k]).max()
    rho = oc.subspace_residual(x_ref, host(Xd), k)
    print(f"PY=2 KH=4 mixed solve: N_chk={k} max|dRitz|={err:.2e} rho={rho:.2e}", flush=True)
    assert err <= 1e-5 and rho <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_projector_terms_in_the_scatter_pass(cs, prec):
    """Every projector term in the separate scatter pass (no stencil-pass records) against
    the oracle, with overlapping supports, and back to the default split."""
    prob = inputs.small_problem(n=(30, 26, 22), h=(0.3, 0.3, 0.3), bc=(0, 0, 1), fd_order=12, n_atoms=9,
                                nproj_per_atom=4, seed=23)
    ns = 6
    dt = "float64" if prec == "fp64" else "float32"
    X = np.random.default_rng(8).standard_normal((prob.nd, ns)).astype(dt)
    ref = apply_h(prob, X.astype(np.float64))
    scale = stencil_scale(prob) * np.abs(X).max()
    tol = 1e-12 * scale if prec == "fp64" else 2e-6 * scale
    h = cs.Handle(prob, precision=cs.FP64 if prec == "fp64" else cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    outs = []
    for in_stencil in (False, True, False):
        h.chefsi_set_projector_pass(in_stencil)
        Yd = torch.zeros(ns, prob.nd, dtype=getattr(torch, dt), device="cuda")
        h.chefsi_apply_h(dev(X, dt), Yd, ns, ws)
        torch.cuda.synchronize()
        got = host(Yd)
        assert np.abs(got - ref).max() <= tol
        outs.append(got)
    assert np.array_equal(outs[0], outs[2])
    assert np.abs(outs[0] - outs[1]).max() <= (1e-13 if prec == "fp64" else 1e-6) * scale


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_keeps_x_and_parity(cs, prec):
    """chefsi_autotune times the candidate tilings and projector splits on the caller's
    block without changing it; H X in the chosen configuration matches the oracle."""
    prob = inputs.small_problem(n=(40, 23, 18), h=(0.3, 0.27, 0.33), bc=(0, 1, 1), fd_order=12, n_atoms=6,
                                nproj_per_atom=4, seed=81)
    ns = 7
    dt = "float64" if prec == "fp64" else "float32"
    X = np.random.default_rng(9).standard_normal((prob.nd, ns)).astype(dt)
    ref = apply_h(prob, X.astype(np.float64))
    scale = stencil_scale(prob) * np.abs(X).max()
    tol = 1e-12 * scale if prec == "fp64" else 2e-6 * scale
    h = cs.Handle(prob, precision=cs.FP64 if prec == "fp64" else cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    Xd = dev(X, dt)
    py, nyg, in_stencil = h.chefsi_autotune(Xd, ns, ws)
    torch.cuda.synchronize()
    print(f"{prec}: autotune chose PY={py} groups={nyg} in_stencil={in_stencil}", flush=True)
    assert np.array_equal(host(Xd), X.astype(np.float64))
    t = h.chefsi_get_stencil_tiling()
    assert (t[0], t[1]) == (py, nyg)
    Yd = torch.zeros_like(Xd)
    h.chefsi_apply_h(Xd, Yd, ns, ws)
    torch.cuda.synchronize()
    assert np.abs(host(Yd) - ref).max() <= tol


def test_band_pass_step_and_solve(cs):
    """Every projector term in the band pass, carried between the filter's applications
    (the coefficients of each application's output come from the same pass): an FP64 step
    against the oracle's, bitwise repeatable, and a mixed solve against the oracle."""
    prob = inputs.small_problem(n=(26, 22, 30), h=(0.3, 0.3, 0.3), bc=(0, 0, 1), fd_order=12, n_atoms=10,
                                nproj_per_atom=4, seed=31)
    ns, degree = 20, 9
    x0 = inputs.initial_block(prob.nd, ns, 5).T
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, x_ref = oc.chefsi_step(prob, x0, degree, lo, cut, hi)
    h = cs.Handle(prob, precision=cs.FP64, max_ns=ns)
    h.chefsi_set_projector_pass(False)
    ws = cs.workspace(h, ns)
    outs = []
    for _ in range(2):
        Xd = dev(x0)
        d = h.chefsi_step(Xd, ns, degree, lo, cut, hi, ws)
        torch.cuda.synchronize()
        outs.append((d, host(Xd)))
    assert np.abs(outs[0][0] - d_ref).max() <= 1e-10
    k = oc.gap_index(d_ref, 16)
    assert oc.subspace_residual(x_ref, outs[0][1], k) <= 1e-8
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    h.close()
    # mixed: n_iter - 1 mixed steps + the FP64 refinement, against the oracle's n_iter steps
    n_iter = 5
    d_ref, x_ref = oc.chefsi(prob, x0, degree, n_iter, lo, cut, hi)
    hm = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    hm.chefsi_set_projector_pass(False)
    wsm = cs.workspace(hm, ns)
    Xm = dev(x0, "float32")
    d, _, _ = hm.solve(Xm, ns, degree, n_iter, wsm, bounds=(lo, cut, hi))
    k = oc.gap_index(d_ref, int(ns / 1.2))
    assert np.abs(d[:k] - d_ref[:k]).max() <= 1e-5
    assert oc.subspace_residual(x_ref, host(Xm), k) <= 1e-5


def test_point_in_too_many_supports_keeps_the_record_route(cs):
    """40 atoms x 4 projectors around one point (160 projector entries there, above the 128
    projectors a band region holds): asking for the band pass is refused and leaves the
    handle on the record route (H X still the oracle's), and autotune keeps the records."""
    n, hh, bc = (16, 16, 16), (0.3, 0.3, 0.3), (0, 0, 0)
    center = np.array([8.0, 8.0, 8.0]) * 0.3
    rng = np.random.Generator(np.random.PCG64(77))
    atoms = center + rng.uniform(-0.25, 0.25, size=(40, 3))
    sp, si, npj, chi, gam = inputs.kb_projectors(n, hh, bc, atoms, 4)
    veff = inputs.gaussian_wells(n, hh, bc, atoms)
    prob = inputs.Problem(n, hh, bc, 12, veff, atoms, sp, si, npj, chi, gam, name="crowded")
    cnt = np.bincount(si, weights=np.repeat(npj, np.diff(sp)), minlength=prob.nd)
    assert cnt.max() > 128
    ns = 6
    x = inputs.initial_block(prob.nd, ns, 3).T
    ref = apply_h(prob, x)
    h = cs.Handle(prob, precision=cs.FP64, max_ns=ns)
    ws = cs.workspace(h, ns)

    def check():
        Y = torch.zeros((ns, prob.nd), dtype=torch.float64, device="cuda")
        h.chefsi_apply_h(dev(x), Y, ns, ws)
        err = np.abs(host(Y) - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, err

    with pytest.raises(cs.ChefsiError, match="too many projector supports"):
        h.chefsi_set_projector_pass(False)
    check()
    py, nyg, in_stencil = h.chefsi_autotune(dev(x), ns, ws)
    print(f"autotune on the crowded grid: rows {py} x groups {nyg}, records {in_stencil}", flush=True)
    assert in_stencil
    check()
    h.close()


def test_autotune_skips_tilings_too_tall_for_the_records(cs):
    """1800 atoms x 4 projectors on a 64 x 64 x 32 grid: the block's projector row (7200
    coefficients) leaves no LDS for the records of the tallest four-rows-per-thread tiles.
    Asking for such a tiling on the record route is refused (the tiling is kept); autotune
    times only the tilings that fit each route and ends with H X still the oracle's; on the
    band pass the tall tiling is accepted, and the record route is then refused with the
    handle left on the band pass."""
    prob = inputs.small_problem(n=(64, 64, 32), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), fd_order=12, n_atoms=1800,
                                nproj_per_atom=4, seed=3)
    assert int(prob.nproj.sum()) == 7200
    ns = 4
    X = np.random.default_rng(10).standard_normal((prob.nd, ns)).astype(np.float32)
    ref = apply_h(prob, X.astype(np.float64))
    tol = 2e-6 * stencil_scale(prob) * np.abs(X).max() + 1e-5 * np.abs(ref).max()
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)

    def check():
        Y = torch.zeros((ns, prob.nd), dtype=torch.float32, device="cuda")
        h.chefsi_apply_h(dev(X, "float32"), Y, ns, ws)
        torch.cuda.synchronize()
        err = np.abs(host(Y) - ref).max()
        assert err <= tol, (err, tol)

    default = h.chefsi_get_stencil_tiling()
    for tall in ((4, 8), (4, 7)):
        with pytest.raises(cs.ChefsiError, match="does not fit in LDS"):
            h.chefsi_set_stencil_tiling(*tall)
        assert h.chefsi_get_stencil_tiling() == default
    check()
    py, nyg, in_stencil = h.chefsi_autotune(dev(X, "float32"), ns, ws)
    print(f"autotune with 7200 projectors: rows {py} x groups {nyg}, records {in_stencil}", flush=True)
    check()
    h.chefsi_set_projector_pass(False)
    h.chefsi_set_stencil_tiling(4, 8)
    check()
    with pytest.raises(cs.ChefsiError, match="does not fit in LDS"):
        h.chefsi_set_projector_pass(True)
    assert h.chefsi_get_stencil_tiling()[:2] == (4, 8)
    check()
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_many_projectors_start_on_the_band_pass(cs, prec):
    """1700 atoms x 4 projectors on a 120 x 120 x 40 slab (at most 14 atoms share a point).
    In FP64 the block's coefficient row (6800 values) leaves no LDS for the record route
    beside any tile of a 120-wide grid: the handle starts on the band pass with H X the
    oracle's, asking for the record route is refused, and autotune stays on the band pass.
    In FP32 the tiles are small enough for the records: the handle starts on the record
    route and autotune may pick either; H X is the oracle's throughout."""
    prob = inputs.small_problem(n=(120, 120, 40), h=(0.3, 0.3, 0.3), bc=(0, 0, 1), fd_order=12, n_atoms=1700,
                                nproj_per_atom=4, seed=41)
    assert int(prob.nproj.sum()) == 6800
    ns = 2
    dt = "float64" if prec == "fp64" else "float32"
    X = np.random.default_rng(12).standard_normal((prob.nd, ns)).astype(dt)
    ref = apply_h(prob, X.astype(np.float64))
    scale = stencil_scale(prob) * np.abs(X).max()
    tol = 1e-12 * scale if prec == "fp64" else 2e-6 * scale + 1e-5 * np.abs(ref).max()
    h = cs.Handle(prob, precision=cs.FP64 if prec == "fp64" else cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)

    def check():
        Y = torch.zeros((ns, prob.nd), dtype=getattr(torch, dt), device="cuda")
        h.chefsi_apply_h(dev(X, dt), Y, ns, ws)
        torch.cuda.synchronize()
        err = np.abs(host(Y) - ref).max()
        assert err <= tol, (err, tol)

    check()
    if prec == "fp64":
        with pytest.raises(cs.ChefsiError, match="does not fit in LDS"):
            h.chefsi_set_projector_pass(True)
        check()
    py, nyg, in_stencil = h.chefsi_autotune(dev(X, dt), ns, ws)
    print(f"{prec}, 6800 projectors: rows {py} x groups {nyg}, records {in_stencil}", flush=True)
    if prec == "fp64":
        assert not in_stencil
    check()
    h.close()
