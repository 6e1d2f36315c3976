"""The request loop on the GPU: every request's result is the same alone and in the
mix within the stated mixed-precision tolerance (1e-5 Ha; the runs are normally
bitwise equal since every kernel here sums in a fixed order, which the test reports),
and a request solved through the loop matches the FP64 oracle."""
import numpy as np
import pytest

from oracle import chefsi as oc
from paper_2302_09708_amd import inputs
from paper_2302_09708_amd.serving import Request, Scheduler, summarize

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    from paper_2302_09708_amd import chefsi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    chefsi.load()
    return chefsi


def _requests(ks, n_iter):
    out = []
    for k in ks:
        prob, ns, degree, seed = inputs.serving_request(k)
        out.append(Request(rid=k, prob=prob, ns=ns, degree=degree, n_iter=n_iter, x_seed=seed, arrival=0.0))
    return out


def test_alone_equals_mix(cs):
    from paper_2302_09708_amd.serving import gpu_ops
    reqs = _requests(range(6), n_iter=4)
    print("requests (N, ns, bc):", [(r.prob.n[0], r.ns, r.prob.bc[2]) for r in reqs], flush=True)
    budget = 8 << 30
    o, r, c = gpu_ops(cs.MIXED)
    alone = Scheduler(budget, 1, o, r, c).run(reqs)
    sched = Scheduler(budget, 4, o, r, c)
    mix = sched.run(reqs)
    assert sched.peak_active > 1          # the solves did run side by side
    worst = 0.0
    for a, m in zip(alone, mix):
        assert a.rid == m.rid
        worst = max(worst, float(np.abs(a.output - m.output).max()))
        assert np.all(np.diff(a.output) >= 0)
    bitwise = all(np.array_equal(a.output, m.output) for a, m in zip(alone, mix))
    print(f"alone vs mix: max |dRitz| = {worst:.3e} Ha (bitwise equal: {bitwise}); mix summary {summarize(mix)}",
          flush=True)
    assert worst <= 1e-5


def test_admission_by_footprint_on_device(cs):
    """A budget that holds only the largest request admits the others around it, never above budget."""
    from paper_2302_09708_amd.serving import gpu_ops
    reqs = _requests(range(4), n_iter=2)
    o, r, c = gpu_ops(cs.MIXED)
    fps = []
    for q in reqs:
        st, fp = o(q)
        fps.append(fp)
        c(st)
    sched = Scheduler(max(fps), 4, o, r, c)
    res = sched.run(reqs)
    assert sched.peak_bytes <= max(fps)
    assert len(res) == 4


def test_request_through_loop_matches_oracle(cs):
    from paper_2302_09708_amd.serving import gpu_ops
    cfg = inputs.CONFIGS["cfg1"]
    prob = inputs.make_problem(cfg)
    x0 = inputs.initial_block(prob.nd, cfg.ns, cfg.x_seed)
    lo, cut, hi = oc.spectral_bounds(prob)
    d_ref, _ = oc.chefsi(prob, x0.T, cfg.degree, cfg.n_iter, lo, cut, hi)
    req = Request(rid=0, prob=prob, ns=cfg.ns, degree=cfg.degree, n_iter=cfg.n_iter, x_seed=cfg.x_seed,
                  arrival=0.0, x0=x0)
    o, r, c = gpu_ops(cs.MIXED)
    res = Scheduler(4 << 30, 2, o, r, c).run([req])
    k = oc.gap_index(d_ref, int(cfg.ns / 1.2))
    err = np.abs(res[0].output[:k] - d_ref[:k]).max()
    print("cfg1 through the loop (mixed, refined): max |dRitz| =", err, flush=True)
    assert err <= 1e-5
