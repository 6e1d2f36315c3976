"""Parity of the complex (Bloch wavevector) path with the complex FP64 oracle through the
C-ABI: H_k X element by element (1e-12 of max |H_k X|) on small grids and on sampled
columns at the bench's full size, one CheFSI step (Ritz values to 1e-10 relative, the
rotated subspace to 1e-8), convergence to the dense spectrum of H_k, k = 0 against the real
handle, argument errors, and bitwise repeatability."""
import numpy as np
import pytest

from oracle import kpoint as ok
from oracle.chefsi import gap_index
from paper_2302_09708_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


CASES = [
    # name, problem arguments, k (bohr^-1)
    ("periodic", dict(n=(16, 15, 14), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), n_atoms=6, nproj_per_atom=4, seed=21),
     (0.4, -0.7, 0.25)),
    ("slab", dict(n=(13, 12, 21), h=(0.3, 0.32, 0.3), bc=(0, 0, 1), n_atoms=4, nproj_per_atom=4, seed=22),
     (-0.9, 0.35, 0.6)),
    ("order4_ragged", dict(n=(17, 11, 13), h=(0.3, 0.35, 0.33), bc=(0, 1, 0), fd_order=4, n_atoms=3,
                           nproj_per_atom=1, seed=23), (1.3, 0.0, -0.45)),
    # 40 wide: tiles of 12 rows, so 29 rows are three tiles with a ragged last one (rows past
    # ny carry the y phase, or are zeros with a Dirichlet y), and the z march runs in chunks
    ("tiles_periodic", dict(n=(40, 29, 18), h=(0.3, 0.31, 0.29), bc=(0, 0, 0), n_atoms=5, nproj_per_atom=4,
                            seed=24), (0.55, -1.1, 0.8)),
    ("tiles_dirichlet_xy", dict(n=(40, 29, 18), h=(0.3, 0.31, 0.29), bc=(1, 1, 0), n_atoms=5, nproj_per_atom=4,
                                seed=25), (0.0, 0.0, -0.6)),
]


def _dev(x):
    """(Nd, ns) complex host array -> (ns, Nd) complex128 device tensor (column-major Nd x ns)."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex128).T)).cuda()


def _host(t):
    return t.detach().cpu().numpy().T.copy()


def _block(nd, ns, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nd, ns)) + 1j * rng.standard_normal((nd, ns))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_apply_h_matches_oracle(cs, case):
    _, args, k = case
    prob = inputs.small_problem(**args)
    img = inputs.support_images(prob)
    ns = 5
    x = _block(prob.nd, ns, 1)
    ref = ok.apply_h_k(prob, img, k, x)
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    X, Y = _dev(x), torch.zeros((ns, prob.nd), dtype=torch.complex128, device="cuda")
    print(f"apply_h {case[0]} n={prob.n} k={k}", flush=True)
    h.apply_h(X, Y, ns, ws)
    y = _host(Y)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"  max rel err {err:.2e}", flush=True)
    assert err < 1e-12
    h.close()


def test_k0_matches_real_handle(cs):
    prob = inputs.small_problem(**CASES[0][1])
    img = inputs.support_images(prob)
    ns = 4
    x = np.random.default_rng(4).standard_normal((prob.nd, ns))
    hk = cs.KPoint(prob, (0.0, 0.0, 0.0), img, max_ns=ns)
    Y = torch.zeros((ns, prob.nd), dtype=torch.complex128, device="cuda")
    hk.apply_h(_dev(x + 0j), Y, ns, hk.workspace(ns))
    hr = cs.Handle(prob, precision=cs.FP64, max_ns=ns)
    Xr = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    Yr = torch.zeros_like(Xr)
    hr.chefsi_apply_h(Xr, Yr, ns, cs.workspace(hr, ns))
    y, yr = _host(Y), _host(Yr)
    assert np.abs(y.imag).max() == 0.0
    assert np.abs(y.real - yr).max() < 1e-12 * np.abs(yr).max()


@pytest.mark.parametrize("case", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_step_matches_oracle(cs, case):
    _, args, k = case
    prob = inputs.small_problem(**args)
    img = inputs.support_images(prob)
    ns, degree = 16, 8
    x = _block(prob.nd, ns, 2)
    lo, cut, hi = -3.0, 2.0, 200.0
    d_ref, x_ref = ok.chefsi_step_k(prob, img, k, x, degree, lo, cut, hi)
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    X = _dev(x)
    print(f"step {case[0]} n={prob.n} k={k} ns={ns}", flush=True)
    d = h.step(X, ns, degree, lo, cut, hi, ws)
    xg = _host(X)
    assert np.abs(d - d_ref).max() < 1e-10 * np.abs(d_ref).max()
    kk = gap_index(d_ref, ns - 2)
    # the rotated subspace of the first kk Ritz vectors (phases of single vectors are free)
    pg = xg[:, :kk] @ xg[:, :kk].conj().T
    po = x_ref[:, :kk] @ x_ref[:, :kk].conj().T
    assert np.abs(pg - po).max() < 1e-8 * np.abs(po).max()
    # bitwise repeatable
    X2 = _dev(x)
    d2 = h.step(X2, ns, degree, lo, cut, hi, ws)
    assert np.array_equal(d, d2) and torch.equal(X, X2)
    h.close()


def test_steps_converge_to_dense_spectrum(cs):
    prob = inputs.small_problem(n=(12, 11, 12), h=(0.3, 0.3, 0.3), bc=(0, 0, 0), fd_order=6, n_atoms=3,
                                nproj_per_atom=4, seed=24)
    img = inputs.support_images(prob)
    k = (0.6, -0.2, 0.9)
    ev = np.linalg.eigvalsh(ok.dense_h_k(prob, img, k))
    ns = 20
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    X = _dev(_block(prob.nd, ns, 5))
    lo, cut, hi = ev[0] - 0.5, ev[0] + 0.1 * (ev[-1] - ev[0]), ev[-1] + 0.5
    for _ in range(25):
        d = h.step(X, ns, 12, lo, cut, hi, ws)
        lo, cut = d[0], d[-1]
    kk = gap_index(d, 14)
    print(f"converged Ritz vs dense: {np.abs(d[:kk] - ev[:kk]).max():.2e} over {kk}", flush=True)
    assert np.abs(d[:kk] - ev[:kk]).max() < 1e-8
    h.close()


def test_bad_arguments(cs):
    prob = inputs.small_problem(**CASES[0][1])
    img = inputs.support_images(prob)
    with pytest.raises(cs.ChefsiError):
        cs.KPoint(prob, (0.1, float("nan"), 0.0), img, max_ns=4)
    h = cs.KPoint(prob, (0.1, 0.2, 0.3), img, max_ns=4)
    ws = h.workspace(4)
    X = torch.zeros((4, prob.nd), dtype=torch.complex128, device="cuda")
    with pytest.raises(cs.ChefsiError):
        h.step(X, 5, 4, -1.0, 0.0, 10.0, ws)  # ns above max_ns
    with pytest.raises(cs.ChefsiError):
        h.step(X, 4, 4, 1.0, 0.0, 10.0, ws)   # lam_lo above lam_cut
    with pytest.raises(cs.ChefsiError):
        h.apply_h(X, X, 4, ws)                # aliasing
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(cs.ChefsiError):
        h.apply_h(X, torch.zeros_like(X), 4, small)
    h.close()


def test_apply_h_full_size_sampled(cs):
    """The bench's k-point configuration (72^3 grid, 128 atoms x 4 projectors, Ns = 600,
    k_d = pi / (2 L_d)), sampled: three columns of H_k X against the oracle, which acts on
    each column alone."""
    prob = inputs.make_problem(inputs.CONFIGS["cfg2"])
    img = inputs.support_images(prob)
    k = tuple(np.pi / (2.0 * prob.n[d] * prob.h[d]) for d in range(3))
    ns = 600
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    X = torch.randn((ns, prob.nd), generator=g, device="cuda", dtype=torch.complex128)
    Y = torch.empty_like(X)
    print(f"apply_h full size n={prob.n} ns={ns}", flush=True)
    h.apply_h(X, Y, ns, ws)
    torch.cuda.synchronize()
    for j in (0, 299, 599):
        x = X[j].cpu().numpy()
        ref = ok.apply_h_k(prob, img, k, x[:, None])[:, 0]
        y = Y[j].cpu().numpy()
        err = np.abs(y - ref).max() / np.abs(ref).max()
        print(f"  column {j}: max rel err {err:.2e}", flush=True)
        assert err < 1e-12
    h.close()


def test_block_above_2_31_elements(cs):
    """A block of 2^31 complex elements or more (120^3 grid with 1000 atoms x 4 projectors,
    Ns = 1300: 2.25e9 elements, 36 GB): sampled columns of H_k X on both sides of element
    2^31 against the oracle, then one step checked by what holds at any size: X^H X = I and
    X^H H_k X = diag(D), over both row panels of the rotation."""
    prob = inputs.make_problem(inputs.CONFIGS["cfg4"])
    img = inputs.support_images(prob)
    k = tuple(np.pi / (2.0 * prob.n[d] * prob.h[d]) for d in range(3))
    ns = 1300
    assert prob.nd * ns >= 1 << 31
    hr = cs.Handle(prob, precision=cs.FP64, max_ns=1)
    lo, cut, hi = hr.chefsi_spectral_bounds()
    hr.close()
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    g = torch.Generator(device="cuda")
    g.manual_seed(78)
    X = torch.randn((ns, prob.nd), generator=g, device="cuda", dtype=torch.complex128)
    Y = torch.empty_like(X)
    print(f"apply_h above 2^31 n={prob.n} ns={ns}", flush=True)
    h.apply_h(X, Y, ns, ws)
    torch.cuda.synchronize()
    first_high = (1 << 31) // prob.nd  # first column holding element 2^31
    for j in (0, first_high, ns - 1):
        ref = ok.apply_h_k(prob, img, k, X[j].cpu().numpy()[:, None])[:, 0]
        err = np.abs(Y[j].cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"  column {j}: max rel err {err:.2e}", flush=True)
        assert err < 1e-12
    print(f"step above 2^31 degree 4 bounds ({lo:.3f}, {cut:.3f}, {hi:.3f})", flush=True)
    d = h.step(X, ns, 4, lo, cut, hi, ws)
    h.apply_h(X, Y, ns, ws)
    G = torch.zeros((ns, ns), dtype=torch.complex128, device="cuda")
    R = torch.zeros_like(G)
    step = 1 << 17
    for r0 in range(0, prob.nd, step):
        xc = X[:, r0:r0 + step]
        G += xc.conj() @ xc.T.contiguous()
        R += xc.conj() @ Y[:, r0:r0 + step].T.contiguous()
    torch.cuda.synchronize()
    eye = torch.eye(ns, dtype=torch.complex128, device="cuda")
    orth = (G - eye).abs().max().item()
    dd = torch.from_numpy(d).to(device="cuda", dtype=torch.complex128)
    ritz = (R - torch.diag(dd)).abs().max().item() / np.abs(d).max()
    print(f"  |X^H X - I| {orth:.2e}, |X^H H X - D| / |D| {ritz:.2e}", flush=True)
    assert orth < 1e-10
    assert ritz < 1e-10
    h.close()


def test_profile_counts_launches(cs):
    """Per-kernel timing of a k-point handle: one step of degree m records m + 1 stencil
    passes, m + 2 band passes (the gather-only pass on X, one per application), one
    projection, one dense stage and one rotation; an unknown id is refused."""
    prob = inputs.small_problem(**CASES[0][1])
    img = inputs.support_images(prob)
    ns, degree = 8, 6
    h = cs.KPoint(prob, CASES[0][2], img, max_ns=ns)
    ws = h.workspace(ns)
    X = _dev(_block(prob.nd, ns, 9))
    h.profile_enable(True)
    h.profile_reset()
    h.step(X, ns, degree, -3.0, 2.0, 200.0, ws)
    counts = [h.profile_read(i)[1] for i in range(5)]
    times = [h.profile_read(i)[0] for i in range(5)]
    print(f"launch counts {counts}, ms {[round(t, 3) for t in times]}", flush=True)
    assert counts == [degree + 1, degree + 2, 1, 1, 1]
    assert all(t > 0.0 for t in times)
    with pytest.raises(cs.ChefsiError):
        h.profile_read(5)
    h.profile_reset()
    assert h.profile_read(0) == (0.0, 0)
    h.close()
