"""Parity at the largest workload sizes, in the launch configurations the benchmark times
(the oracle computes what it can one column or one entry at a time):

  * H X on the full 120^3 workload (1000 atoms x 4 projectors, Ns = 7200, FP32 block of
    49.8 GB) on sampled columns, mixed handle, default tiling (two rows per thread, four
    halo values: the variant the FP32 filter of that workload runs);
  * the split-bf16 projection with K = Nd = 1.728 M in one chunk: sampled entries against
    FP64 products of the same FP32 data, and against the exact value of the three bf16
    products, which isolates the FP32 summation (FP32 sums span at most 16384 rows before
    they move into FP64);
  * the FP64 Gram products and rotation of a block of more than 2^31 elements
    (Nd = 1.728 M, Ns = 1300; the rotation takes the hand-written FP64 MFMA kernel there),
    on sampled entries and grid points.
"""
import numpy as np
import pytest

from paper_2302_09708_amd import inputs
from tests._gpu import stencil_scale

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


def test_full_size_cfg4_apply_h_sampled(cs):
    from oracle.hamiltonian import apply_h
    cfg = inputs.CONFIGS["cfg4"]
    print("cfg4: building the problem", flush=True)
    prob = inputs.make_problem(cfg)
    ns = cfg.ns
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    print("cfg4: tiling", h.chefsi_get_stencil_tiling(), flush=True)
    ws = cs.workspace(h, ns)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    X = torch.randn(ns, prob.nd, dtype=torch.float32, device="cuda", generator=gen)
    Y = torch.empty_like(X)
    print("cfg4: apply_h on 7200 orbitals", flush=True)
    h.chefsi_apply_h(X, Y, ns, ws)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 1777, 3600, 5123, 7198, 7199]
    xs = X[cols].double().cpu().numpy().T
    got = Y[cols].double().cpu().numpy().T
    del X, Y, ws
    torch.cuda.empty_cache()
    ref = apply_h(prob, xs)
    err = np.abs(got - ref).max()
    scale = stencil_scale(prob) * np.abs(xs).max()
    print(f"cfg4 H X sampled: max err {err:.3e} (scale {scale:.3e})", flush=True)
    assert err <= 2e-6 * scale


def _sample_pairs(ns, rng, k):
    i = rng.integers(0, ns, size=k)
    j = rng.integers(0, ns, size=k)
    diag = np.arange(0, ns, max(1, ns // 16))
    return np.concatenate([i, diag]), np.concatenate([j, diag])


def _bf16_rne(x32):
    """float32 array -> float64 values of its bf16 rounding (round to nearest even)."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _split(x32):
    hi = _bf16_rne(x32)
    lo = _bf16_rne((x32.astype(np.float64) - hi).astype(np.float32))
    return hi, lo


def test_split_bf16_gram_at_k_of_1_7_million(cs):
    """Ns = 5760 is 1035 upper tiles, enough that the projection runs one K chunk of all
    1.728 M rows per tile (the plan of the 120^3, Ns = 7200 workload)."""
    n = (120, 120, 120)
    prob = inputs.small_problem(n=n, h=(0.22, 0.22, 0.22), n_atoms=0, nproj_per_atom=0, seed=1, with_veff=False)
    ns = 5760
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    ws = cs.workspace(h, ns)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    X = torch.randn(ns, prob.nd, dtype=torch.float32, device="cuda", generator=gen)
    X += 0.5  # a common offset: large positive sums, where long FP32 sums lose most
    Hs = torch.zeros(ns, ns, dtype=torch.float64, device="cuda")
    Ms = torch.zeros_like(Hs)
    print("split-bf16 projection, K = 1728000, Ns = 5760", flush=True)
    h.chefsi_project(X, ns, Hs, Ms, ws)
    torch.cuda.synchronize()
    del ws
    rng = np.random.default_rng(3)
    ii, jj = _sample_pairs(ns, rng, 40)
    ms = Ms.cpu().numpy()
    worst_split, worst = 0.0, 0.0
    for i, j in zip(ii, jj):
        a32 = X[i].cpu().numpy()
        b32 = X[j].cpu().numpy()
        a, b = a32.astype(np.float64), b32.astype(np.float64)
        exact = float(a @ b)
        sab = float(np.abs(a) @ np.abs(b))
        ah, al = _split(a32)
        bh, bl = _split(b32)
        # what the three bf16 products give in exact arithmetic (they are exact in FP32)
        split = float(ah @ bh + ah @ bl + al @ bh)
        got = ms[j, i]  # element (i, j) of the column-major result
        # rigorous: representation error of the split, FP32 sums over at most 16384 rows
        assert abs(got - exact) <= (3.1 * U16 + 16384 * U24) * sab
        worst = max(worst, abs(got - exact) / sab)
        worst_split = max(worst_split, abs(got - split) / sab)
    print(f"split-bf16 Gram at K = 1.7M: worst |err| / sum|ab| = {worst:.2e}, "
          f"FP32-summation part {worst_split:.2e}", flush=True)
    # the summation error alone stays far inside the bound (one FP32 sum over all 1.7 M
    # rows would leave ~2e-5 on the offset diagonal)
    assert worst_split <= 2e-6


def test_fp64_gram_and_rotation_above_2_31_elements(cs):
    n = (120, 120, 120)
    prob = inputs.small_problem(n=n, h=(0.22, 0.22, 0.22), n_atoms=0, nproj_per_atom=0, seed=1, with_veff=False)
    ns = 1300
    assert prob.nd * ns >= 2 ** 31
    h = cs.Handle(prob, precision=cs.FP64, max_ns=ns)
    ws = cs.workspace(h, ns)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(6)
    X = torch.randn(ns, prob.nd, dtype=torch.float64, device="cuda", generator=gen)
    Hs = torch.zeros(ns, ns, dtype=torch.float64, device="cuda")
    Ms = torch.zeros_like(Hs)
    print("FP64 projection, Nd = 1728000, Ns = 1300", flush=True)
    h.chefsi_project(X, ns, Hs, Ms, ws)
    torch.cuda.synchronize()
    ms = Ms.cpu().numpy().T
    rng = np.random.default_rng(4)
    ii, jj = _sample_pairs(ns, rng, 32)
    for i, j in zip(ii, jj):
        a = X[i].cpu().numpy()
        b = X[j].cpu().numpy()
        assert abs(ms[i, j] - float(a @ b)) <= 1e-12 * float(np.abs(a) @ np.abs(b))
    # rotation X <- X Z on sampled grid points: O[:, p] = Z^T X[:, p]
    Z = torch.randn(ns, ns, dtype=torch.float64, device="cuda", generator=gen) / np.sqrt(ns)
    pts = torch.tensor([0, 1, 4097, 999_999, prob.nd - 2, prob.nd - 1], device="cuda")
    x_pts = X[:, pts].cpu().numpy()                    # ns x npts
    z = Z.cpu().numpy().T                              # Z column-major in the tensor's transpose
    print("FP64 rotation, Nd = 1728000, Ns = 1300", flush=True)
    h.chefsi_rotate(X, Z, ns, ws)
    torch.cuda.synchronize()
    got = X[:, pts].cpu().numpy()
    ref = z.T @ x_pts
    err = np.abs(got - ref).max()
    print(f"FP64 rotation above 2^31 elements: max err {err:.2e}", flush=True)
    assert err <= 1e-12 * np.abs(z).sum(axis=0).max() * np.abs(x_pts).max()
