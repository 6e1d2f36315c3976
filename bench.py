"""CheFSI step throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2] [--precision fp64|mixed]

A step is one whole CheFSI iteration (Alg. 1: filtering, projection, FP64
subspace diagonalisation, rotation, Ritz values to the host) on one block of
synthetic orbitals already resident in HBM.  The default workload is the
periodic 72^3 grid (h = 0.25 bohr, FD order 12), 128 atoms with s + 3p
Kleinman-Bylander projectors, Ns = 600, Chebyshev degree 20, plain FP64.

Prints ONE JSON line with iterations/s, the roofline position of the dominant
kernel (timed with HIP events recorded by the library on its launch stream),
the other precision on the same inputs ("compare": FP64 vs mixed) and, at
N = 1, the FP64 CPU oracle timed on a bounded sample of the same workload on
this host's cores.  Figures outside the timed steps: the Lanczos estimate of
lambda_Nd, the nonlocal forces, and (72^3 and 24^3 workloads) the same grid at
a Bloch wavevector in complex FP64 ("kpoint").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6      # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TFS = 2500.0    # MI355X dense BF16 matrix
KERNELS = ["hx_apply", "nonlocal", "gram", "gram_reduce", "rotate", "dense_eig", "copy", "fp64_fallback_steps"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hx_apply_cfg2_fp64_traffic.txt")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="cfg2")
    p.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-compare", action="store_true", help="skip the other precision on the same inputs")
    p.add_argument("--requests", type=int, default=256, help="cfg5: number of requests")
    p.add_argument("--slots", type=int, default=4, help="cfg5: concurrent solves")
    p.add_argument("--calibration", type=int, default=16, help="cfg5: requests solved alone to set the rate")
    p.add_argument("--cpu-columns", type=int, default=8)
    p.add_argument("--no-subrecords", action="store_true",
                   help="skip the cfg3/cfg4 mixed and serving records after the headline")
    p.add_argument("--serving-requests", type=int, default=48, help="requests of the serving record")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="after the timed steps, run one plain device copy of 1 GiB (counter calibration)")
    p.add_argument("--gemm-probe", action="store_true",
                   help="only the mixed handle's projection and rotation on the workload's block sizes (no "
                        "dense stage): prints their times and MFMA rates, for counter runs of the split-bf16 kernels")
    p.add_argument("--fixed-stencil", default=None, metavar="PY,GROUPS,IN_STENCIL",
                   help="set this stencil tiling and projector route instead of timing the candidates "
                        "(every run of the invocation; for counter passes that must profile one kernel)")
    return p.parse_args()


def kernel_source_hash(*names: str) -> str:
    """First 16 hex digits of the SHA-256 of the named csrc files, concatenated in order."""
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_2302_09708_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(prob, cfg, ns_cols: int):
    """The FP64 oracle timed on this host on a bounded sample of one CheFSI iteration of
    this workload, on the workload's own inputs (seeded X0):

      * the filter (degree m) and the extra H X~ on ``ns_cols`` of the Ns columns, scaled
        by Ns / ns_cols (the oracle applies H to each column independently, so this cost
        is linear in Ns);
      * the two Gram products, the dense generalized eigensolve and the rotation X~ Z~,
        each run once in full on the whole block (X0 stands in for X~ and Y~, and its
        Gram matrix plus a spread diagonal for H~: these costs do not depend on the
        values);

    plus, for scale, whole oracle iterations of the 24^3 workload (median of five)."""
    from oracle import chefsi as oc
    from paper_2302_09708_amd.inputs import CONFIGS, initial_block, make_problem

    from oracle.hamiltonian import apply_h
    lo, cut, hi = oc.spectral_bounds(prob)
    x = initial_block(prob.nd, cfg.ns, cfg.x_seed).T   # Nd x Ns
    xs = np.ascontiguousarray(x[:, :ns_cols])
    t0 = time.perf_counter()
    xf = oc.chebyshev_filter(prob, xs, cfg.degree, lo, cut, hi)
    apply_h(prob, xf)
    t_filter = (time.perf_counter() - t0) * cfg.ns / ns_cols
    t0 = time.perf_counter()
    hs = x.T @ x
    ms = x.T @ x
    t_proj = time.perf_counter() - t0
    hs = 0.5 * (hs + hs.T) + np.diag(np.arange(cfg.ns, dtype=np.float64))
    ms = 0.5 * (ms + ms.T)
    t0 = time.perf_counter()
    d, z = oc.diagonalize(hs, ms)
    t_eig = time.perf_counter() - t0
    t0 = time.perf_counter()
    oc.rotate(x, z)
    t_rot = time.perf_counter() - t0
    total = t_filter + t_proj + t_eig + t_rot
    # whole iterations of the small workload
    c1 = CONFIGS["cfg1"]
    p1 = make_problem(c1)
    x1 = initial_block(p1.nd, c1.ns, c1.x_seed).T
    l1, k1, h1 = oc.spectral_bounds(p1)
    its = []
    for _ in range(5):
        t0 = time.perf_counter()
        d1, x1 = oc.chefsi_step(p1, x1, c1.degree, l1, k1, h1)
        its.append(time.perf_counter() - t0)
        l1, k1 = float(d1[0]), float(d1[-1])
    cores = len(os.sched_getaffinity(0))
    return {
        "value": 1.0 / total, "unit": "iter/s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle on the {cfg.name} inputs: filter (degree {cfg.degree}) + H X on {ns_cols} of {cfg.ns} "
                   f"columns scaled x{cfg.ns / ns_cols:g} ({t_filter:.1f} s); X^T Y and X^T X on the whole block "
                   f"({t_proj:.1f} s); dsygvd {cfg.ns} ({t_eig:.2f} s); X Z ({t_rot:.2f} s); NumPy stencil "
                   f"single-threaded, BLAS/LAPACK on {cores} threads; 24^3 workload whole iterations, median of 5"),
        "seconds_per_iter": total,
        "cfg1_whole_iter_per_s": 1.0 / float(np.median(its)),
    }


def gram_block_starts(ns: int) -> list:
    """Column blocks of the library's upper-triangle FP64 Gram (block row q is formed
    against columns start_q .. ns - 1 only): 128 wide up to ns = 1024, else three blocks
    cut near 0.43 ns and 0.75 ns."""
    if ns < 256:
        return [0, ns]
    if ns <= 1024:
        return list(range(0, ns, 128)) + [ns]
    return [0, int(0.43 * ns / 128 + 0.5) * 128, int(0.75 * ns / 128 + 0.5) * 128, ns]


def gemm_figures(nd: int, ns: int, prec: int, gram_ms: float, rot_ms: float, fp64: bool):
    """Algorithmic and executed MFMA flops of one step's projection (two Gram products) and rotation."""
    alg = 2.0 * nd * ns * (ns + 1) * 2 + 2.0 * nd * ns * ns
    nt = (ns + 127) // 128
    if fp64:
        b = gram_block_starts(ns)                                     # rocBLAS dgemm per column block
        gram_exec = 2 * sum(2.0 * nd * (b[q + 1] - b[q]) * (ns - b[q]) for q in range(len(b) - 1))
        rot_exec = 2.0 * nd * ns * ns
        mult, peak, unit_dtype = 1, FP64_MFMA_PEAK_TFS, "f64"
    else:
        ld = (ns + 31) // 32 * 32
        cols = (ns + 127) // 128 * 128
        rot_exec = 2.0 * ((nd + 255) // 256 * 256) * cols * ld
        gram_exec = 2 * (2.0 * nd * 128 * 128 * nt * (nt + 1) // 2)  # upper 128 x 128 tiles only
        mult, peak, unit_dtype = 3, BF16_MFMA_PEAK_TFS, "bf16"   # three bf16 products per FP32 product
    t = (gram_ms + rot_ms) * 1e-3
    executed = mult * (gram_exec + rot_exec)
    return {"algorithmic_tflops": alg / t / 1e12, "executed_tflops": executed / t / 1e12, "mfma_dtype": unit_dtype,
            "peak_tflops": peak, "utilisation": executed / t / 1e12 / peak,
            "gram_executed_tflops": mult * gram_exec / (gram_ms * 1e-3) / 1e12,
            "rotate_executed_tflops": mult * rot_exec / (rot_ms * 1e-3) / 1e12}


def initial_device_block(prob, cfg, tdt, x0):
    """X0 on the device: the seeded NumPy block when given, else (blocks too large to draw on
    the host in reasonable time) torch's seeded N(0,1) in FP32 on the device, widened for FP64."""
    import torch
    if x0 is not None:
        return torch.from_numpy(x0).to(device="cuda", dtype=tdt)
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.x_seed)
    X = torch.randn((cfg.ns, prob.nd), generator=g, device="cuda", dtype=torch.float32)
    return X if tdt == torch.float32 else X.to(tdt)


FIXED_STENCIL = None  # (rows per thread, row groups, projectors in the stencil pass) from --fixed-stencil


def gemm_probe(args):
    """The mixed handle's projection (Hs = X^T H X, Ms = X^T X: one stencil pass and the two
    split-bf16 Gram products) and rotation (X <- X Z, Z the identity, so X stays bounded) on
    the workload's Nd x Ns block drawn on the device, `steps` times after one warm-up each,
    timed by the library's HIP events.  No dense stage: for hardware-counter runs of the
    split-bf16 kernels at sizes whose full step cannot run under the counter profiler."""
    import torch
    from paper_2302_09708_amd import chefsi as cs
    from paper_2302_09708_amd import inputs
    cs.load()
    cfg = inputs.CONFIGS[args.workload]
    prob = inputs.make_problem(cfg)
    ns = cfg.ns
    h = cs.Handle(prob, precision=cs.MIXED, max_ns=ns)
    X = initial_device_block(prob, cfg, torch.float32, None)
    ws = cs.workspace(h, ns)
    Hs = torch.empty(ns * ns, dtype=torch.float64, device="cuda")
    Ms = torch.empty_like(Hs)
    Z = torch.eye(ns, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    h.chefsi_project(X, ns, Hs, Ms, ws, stream=stream)
    h.chefsi_rotate(X, Z, ns, ws, stream=stream)
    torch.cuda.synchronize()
    h.chefsi_profile_enable(True)
    h.chefsi_profile_reset()
    for i in range(args.steps):
        h.chefsi_project(X, ns, Hs, Ms, ws, stream=stream)
        h.chefsi_rotate(X, Z, ns, ws, stream=stream)
        print(f"[gemm-probe] {cfg.name} call {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    kern = {}
    for kid, name in enumerate(KERNELS):
        ms, n = h.chefsi_profile_read(kid)
        kern[name] = ms / args.steps
    h.chefsi_profile_enable(False)
    g = gemm_figures(prob.nd, ns, cs.MIXED, kern["gram"] + kern["gram_reduce"], kern["rotate"], False)
    print(json.dumps({"mode": "gemm_probe", "workload": cfg.name, "nd": prob.nd, "ns": ns, "calls": args.steps,
                      "ms_per_call": {k: v for k, v in kern.items() if v > 0}, "gemm": g}))
    h.close()


def run_path(cs, prob, cfg, precision: str, steps: int, warmup: int, x0):
    """Time `steps` CheFSI steps of one precision on the workload; per-kernel HIP-event times."""
    import torch
    prec = cs.FP64 if precision == "fp64" else cs.MIXED
    tdt = torch.float64 if prec == cs.FP64 else torch.float32
    ns, m = cfg.ns, cfg.degree
    h = cs.Handle(prob, precision=prec, max_ns=ns)
    X = initial_device_block(prob, cfg, tdt, x0)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ws = cs.workspace(h, ns)
    lo, cut, hi = h.chefsi_spectral_bounds()
    stream = torch.cuda.current_stream()
    # one-time set-up: stencil tiling and projector split picked by timing (X is not changed)
    t_tune = time.perf_counter()
    if FIXED_STENCIL is None:
        tuned = h.chefsi_autotune(X, ns, ws, stream=stream)
    else:
        h.chefsi_set_projector_pass(bool(FIXED_STENCIL[2]))
        h.chefsi_set_stencil_tiling(FIXED_STENCIL[0], FIXED_STENCIL[1])
        tuned = FIXED_STENCIL
    tune_s = time.perf_counter() - t_tune
    for _ in range(warmup):
        d = h.chefsi_step(X, ns, m, lo, cut, hi, ws, stream=stream)
        lo, cut = float(d[0]), float(d[-1])
    torch.cuda.synchronize()
    h.chefsi_profile_enable(True)
    h.chefsi_profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        d = h.chefsi_step(X, ns, m, lo, cut, hi, ws, stream=stream)
        lo, cut = float(d[0]), float(d[-1])
        print(f"[bench] {precision} step {i + 1}/{steps} D1={d[0]:.6f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern = {}
    for kid, name in enumerate(KERNELS):
        ms, n = h.chefsi_profile_read(kid)
        kern[name] = {"ms_per_step": ms / steps, "launches_per_step": n / steps, "avg_launch_ms": ms / n if n else 0.0}
    h.chefsi_profile_reset()
    ritz_steps = d
    fallback_steps = kern["fp64_fallback_steps"]["launches_per_step"] * steps
    refine_ms = None
    ritz_refined = None
    if prec == cs.MIXED:  # the once-per-solve FP64 refinement (filter + FP64 Rayleigh-Ritz), timed once
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ritz_refined = h.chefsi_refine_fp64(X, ns, ws, m, lo, cut, hi, stream=stream)
        torch.cuda.synchronize()
        refine_ms = (time.perf_counter() - t1) * 1e3
    h.chefsi_profile_enable(False)
    del X, ws
    h.close()
    torch.cuda.empty_cache()
    b = 8 if prec == cs.FP64 else 4
    hx_bytes_step = (3 * m + 1) * prob.nd * ns * b + (m + 1) * prob.nd * b
    hx_ms = kern["hx_apply"]["ms_per_step"]
    out = {"precision": precision, "iter_per_s": steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
           "hx_gbs": hx_bytes_step / (hx_ms * 1e-3) / 1e9, "hx_bytes_step": hx_bytes_step, "kernels": kern,
           "gemm": gemm_figures(prob.nd, ns, prec, kern["gram"]["ms_per_step"] + kern["gram_reduce"]["ms_per_step"],
                                kern["rotate"]["ms_per_step"], prec == cs.FP64)}
    out["ritz_steps"] = ritz_steps
    out["stencil_choice"] = {"rows_per_thread": tuned[0], "row_groups": tuned[1], "projectors_in_stencil": tuned[2],
                             "autotune_s": tune_s if FIXED_STENCIL is None else None}
    out["fallback_steps"] = int(round(fallback_steps))
    if refine_ms is not None:
        out["refine_ms"] = refine_ms
        out["ritz_refined"] = ritz_refined
        # a solve of n_iter filter passes: n_iter - 1 mixed steps + the refinement
        out["solve_ms"] = (cfg.n_iter - 1) * out["ms_per_step"] + refine_ms
    else:
        out["solve_ms"] = cfg.n_iter * out["ms_per_step"]
    return out


def lanczos_figures(cs, prob, cfg, precision: str, steps: int = 20):
    """Device Lanczos estimate of lam_Nd on the workload (outside the timed steps): time of
    `steps` steps, the estimate and the Gershgorin bound the timed steps start from."""
    import torch
    from paper_2302_09708_amd import inputs
    prec = cs.FP64 if precision == "fp64" else cs.MIXED
    h = cs.Handle(prob, precision=prec, max_ns=1)
    ws = torch.empty(h.chefsi_lanczos_workspace_bytes(), dtype=torch.uint8, device="cuda")
    v = torch.from_numpy(inputs.initial_block(prob.nd, 1, cfg.x_seed + 1)[0]).to(
        device="cuda", dtype=torch.float64 if prec == cs.FP64 else torch.float32)
    h.chefsi_lanczos_bound(v, steps, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, theta, _, _ = h.chefsi_lanczos_bound(v, steps, ws)
    ms = (time.perf_counter() - t0) * 1e3
    gersh = h.chefsi_spectral_bounds()[2]
    h.close()
    del ws, v
    torch.cuda.empty_cache()
    return {"steps": steps, "ms": ms, "theta": theta, "lam_nd": lam, "gershgorin_lam_hi": gersh}


def forces_figures(cs, prob, cfg, precision: str):
    """Nonlocal forces of the workload's Ns orbitals (outside the timed steps): time of one
    call (three gradient passes, four projector gathers, the force sums)."""
    import torch
    prec = cs.FP64 if precision == "fp64" else cs.MIXED
    ns = cfg.ns
    h = cs.Handle(prob, precision=prec, max_ns=ns)
    ws = torch.empty(h.chefsi_forces_workspace_bytes(ns), dtype=torch.uint8, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.x_seed + 2)
    X = torch.randn((ns, prob.nd), generator=g, device="cuda",
                    dtype=torch.float64 if prec == cs.FP64 else torch.float32)
    occ = np.full(ns, 2.0)
    h.chefsi_nonlocal_forces(X, ns, occ, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = h.chefsi_nonlocal_forces(X, ns, occ, ws)
    ms = (time.perf_counter() - t0) * 1e3
    h.close()
    del ws, X
    torch.cuda.empty_cache()
    return {"ms": ms, "atoms": int(f.shape[0]), "orbitals": ns, "max_abs_force": float(np.abs(f).max())}


def kpoint_figures(cs, prob, cfg):
    """The workload's grid, atoms and Ns at the Bloch wavevector k_d = pi / (2 L_d) in
    complex FP64 (outside the timed steps): step rate, per-kernel milliseconds per step
    (HIP events the library records on the launch stream), the stencil pass's own rate, and
    the rate of one whole H_k application (coefficient gather, Bloch-phased stencil,
    projector scatter) counted on the stencil's bytes."""
    import torch
    from paper_2302_09708_amd import inputs
    ns, m = cfg.ns, cfg.degree
    k = tuple(np.pi / (2.0 * prob.n[d] * prob.h[d]) for d in range(3))
    img = inputs.support_images(prob)
    hr = cs.Handle(prob, precision=cs.FP64, max_ns=1)
    lo, cut, hi = hr.chefsi_spectral_bounds()
    hr.close()
    h = cs.KPoint(prob, k, img, max_ns=ns)
    ws = h.workspace(ns)
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg.x_seed + 3)
    X = torch.randn((ns, prob.nd), generator=g, device="cuda", dtype=torch.complex128)
    Y = torch.empty_like(X)
    h.apply_h(X, Y, ns, ws)
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    b.record()
    for _ in range(reps):
        h.apply_h(X, Y, ns, ws)
    e.record()
    torch.cuda.synchronize()
    apply_ms = b.elapsed_time(e) / reps
    del Y
    d = h.step(X, ns, m, lo, cut, hi, ws)  # warm-up step
    lo, cut = d[0], d[-1]
    steps = 2
    h.profile_reset()
    h.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        d = h.step(X, ns, m, lo, cut, hi, ws)
        lo, cut = d[0], d[-1]
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / steps
    names = ("zhx", "band", "gram", "dense_eig", "rotate")
    per_kernel = {}
    for i, name in enumerate(names):
        ms, n = h.profile_read(i)
        per_kernel[name] = {"ms_per_step": ms / steps, "launches_per_step": n / steps}
    h.close()
    # the stencil pass's own rate: (3m+1) complex arrays of Nd x Ns move per step (the first
    # filter pass and the pass forming H X~ read one and write one, the others read two and
    # write one) plus Veff per launch, over the summed zhx launch time
    zhx_bytes = 16.0 * prob.nd * ns * (3 * m + 1) + 8.0 * prob.nd * (m + 1)
    zhx_gbs = zhx_bytes / (per_kernel["zhx"]["ms_per_step"] * 1e-3) / 1e9
    del X, ws
    torch.cuda.empty_cache()
    # algorithmic bytes of one application: read X, write Y (16 B each per point and
    # orbital), Veff once, the projector values and alpha (small)
    apply_bytes = prob.nd * ns * 32.0 + prob.nd * 8.0
    gbs = apply_bytes / (apply_ms * 1e-3) / 1e9
    return {"k_bohr_inv": list(k), "dtype": "c128", "iter_per_s": 1e3 / step_ms, "ms_per_step": step_ms,
            "kernels": per_kernel, "zhx_gbs": zhx_gbs, "zhx_frac": zhx_gbs / HBM_PEAK_GBS,
            "apply_h_ms": apply_ms, "apply_h_gbs": gbs, "apply_h_frac": gbs / HBM_PEAK_GBS,
            "ritz_lowest": float(d[0])}


def copy_gbs():
    """Bandwidth of a plain 1 GiB device-to-device copy (read + write bytes / time), the
    practical streaming ceiling the stencil's rate is also compared with."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / best / 1e9


def serving_bench(args):
    """Serving stream: Poisson arrivals of CheFSI solve requests of mixed sizes, continuous
    admission by slot and HBM footprint; p50/p99 latency and solves/s."""
    import torch
    from paper_2302_09708_amd import chefsi as cs
    from paper_2302_09708_amd import inputs, serving

    n_req = args.requests
    t0 = time.perf_counter()
    specs = []
    for k in range(n_req):
        prob, ns, degree, seed = inputs.serving_request(k)
        specs.append((prob, ns, degree, seed))
        if (k + 1) % 32 == 0:
            print(f"[bench] generated {k + 1}/{n_req} requests ({time.perf_counter() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    o, r, c = serving.gpu_ops(cs.MIXED)

    def reqs(idx, arrivals):
        return [serving.Request(rid=k, prob=specs[k][0], ns=specs[k][1], degree=specs[k][2], n_iter=10,
                                x_seed=specs[k][3], arrival=float(a)) for k, a in zip(idx, arrivals)]

    # warm-up and calibration: requests solved alone, one after another
    serving.Scheduler(budget, 1, o, r, c).run(reqs([0], [0.0]))
    n_cal = min(args.calibration, n_req)
    cal = serving.Scheduler(budget, 1, o, r, c).run(reqs(range(n_cal), [0.0] * n_cal))
    solo = float(np.mean([x.finished - x.admitted for x in cal]))
    rate = 0.8 / solo
    print(f"[bench] mean solo solve {solo * 1e3:.1f} ms -> arrival rate {rate:.2f}/s", file=sys.stderr, flush=True)
    arrivals = serving.poisson_arrivals(n_req, rate, seed=5000)
    sched = serving.Scheduler(budget, args.slots, o, r, c, fail_fast=False)
    res = sched.run(reqs(range(n_req), arrivals))
    for x in res:
        if x.error is not None:
            print(f"[bench] request {x.rid} failed: {x.error}", file=sys.stderr, flush=True)
    st = serving.summarize(res)
    out = {
        "metric": "serving solves/s", "value": st["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32+bf16x3+f64", "data": "synthetic",
        "config": {"workload": f"cfg5: {n_req} requests, Poisson arrivals at 0.8 / mean solo solve time, "
                               "cubic N ~ U{24..64}, h 0.3, 8-96 atoms x 4 projectors, Ns ~ U{40..400}, "
                               "periodic or Dirichlet-z slab 50/50, degree 20, 10 iterations (9 mixed + refine)",
                   "slots": args.slots, "hbm_budget_bytes": budget},
        "p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_latency_s": st["mean_s"], "makespan_s": st["makespan_s"],
        "failed_requests": st["failed"],
        "mean_solo_solve_s": solo, "arrival_rate_per_s": rate, "peak_admitted_bytes": sched.peak_bytes,
        "peak_concurrent": sched.peak_active,
    }
    print(json.dumps(out), flush=True)


def workload_record(cs, name: str, steps: int, warmup: int, with_fp64: bool):
    """A mixed-precision workload outside the headline's timed region: per-step time and
    kernel split, stencil rate, split-bf16 MFMA utilisation, FP64 fallbacks, the FP64
    refinement and how far it moves the Ritz values; optionally the FP64 path on the same
    (device-drawn) X0."""
    import torch
    from paper_2302_09708_amd import inputs
    cfg = inputs.CONFIGS[name]
    t0 = time.perf_counter()
    prob = inputs.make_problem(cfg)
    setup_s = time.perf_counter() - t0
    print(f"[bench] {name}: Nd={prob.nd} Ns={cfg.ns} mixed ({setup_s:.1f} s to build the problem)",
          file=sys.stderr, flush=True)
    mixed = run_path(cs, prob, cfg, "mixed", steps, warmup, None)
    k_chk = max(1, int(cfg.ns / 1.2))
    moved = np.abs(mixed["ritz_refined"][:k_chk] - mixed["ritz_steps"][:k_chk])
    rec = {
        "workload": f"{name}: {'x'.join(map(str, cfg.n))} grid h={cfg.h[0]}, bc {''.join('PD'[b] for b in cfg.bc)}, "
                    f"{cfg.n_atoms} atoms x {cfg.nproj_per_atom} projectors, Ns={cfg.ns}, degree {cfg.degree}, "
                    f"X0 drawn on the device (seed {cfg.x_seed})",
        "steps": steps, "warmup": warmup,
        "mixed": {"iter_per_s": mixed["iter_per_s"], "ms_per_step": mixed["ms_per_step"],
                  "hx_gbs": mixed["hx_gbs"], "hx_frac": mixed["hx_gbs"] / HBM_PEAK_GBS,
                  "gemm_utilisation": mixed["gemm"]["utilisation"],
                  "gram_executed_tflops": mixed["gemm"]["gram_executed_tflops"],
                  "rotate_executed_tflops": mixed["gemm"]["rotate_executed_tflops"],
                  "kernels_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in mixed["kernels"].items()},
                  "stencil_choice": mixed["stencil_choice"],
                  "fp64_fallback_steps": mixed["fallback_steps"],
                  "refine_ms": mixed["refine_ms"],
                  "ritz_lowest": float(mixed["ritz_refined"][0]),
                  "refine_max_ritz_change_first_nchk": float(moved.max()), "n_chk": k_chk},
    }
    if with_fp64:
        fp = run_path(cs, prob, cfg, "fp64", steps, warmup, None)
        rec["fp64"] = {"iter_per_s": fp["iter_per_s"], "ms_per_step": fp["ms_per_step"], "hx_gbs": fp["hx_gbs"],
                       "gemm_utilisation": fp["gemm"]["utilisation"],
                       "kernels_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in fp["kernels"].items()}}
        rec["mixed_over_fp64_step_speedup"] = mixed["iter_per_s"] / fp["iter_per_s"]
    torch.cuda.empty_cache()
    return rec


def serving_record(args, n_req: int):
    """A short serving stream (the cfg5 recipe with fewer requests) outside the timed steps."""
    import io
    import contextlib
    a = argparse.Namespace(**vars(args))
    a.requests, a.calibration = n_req, min(args.calibration, 8)
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        serving_bench(a)
    r = json.loads(buf.getvalue().strip().splitlines()[-1])
    return {k: r[k] for k in ("value", "unit", "p50_s", "p99_s", "mean_latency_s", "makespan_s", "failed_requests",
                              "mean_solo_solve_s", "arrival_rate_per_s", "peak_concurrent")} | {
        "requests": n_req, "slots": args.slots}


def main():
    global FIXED_STENCIL
    args = parse()
    if args.fixed_stencil:
        FIXED_STENCIL = tuple(int(v) for v in args.fixed_stencil.split(","))
        assert len(FIXED_STENCIL) == 3, "--fixed-stencil takes PY,GROUPS,IN_STENCIL"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is design only",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "cfg5":
        serving_bench(args)
        return
    if args.gemm_probe:
        gemm_probe(args)
        return
    import torch
    from paper_2302_09708_amd import chefsi as cs
    from paper_2302_09708_amd import inputs

    cfg = inputs.CONFIGS[args.workload]
    precision = args.precision or ("fp64" if args.workload in ("cfg1", "cfg2") else "mixed")
    prob = inputs.make_problem(cfg)
    ns, m = cfg.ns, cfg.degree
    print(f"[bench] {cfg.name} Nd={prob.nd} Ns={ns} degree={m} {precision}", file=sys.stderr, flush=True)
    # the seeded NumPy block (as the oracle uses) unless it is too large to draw on the host
    x0 = inputs.initial_block(prob.nd, ns, cfg.x_seed) if prob.nd * ns <= 1_000_000_000 else None
    main_run = run_path(cs, prob, cfg, precision, args.steps, args.warmup, x0)
    other = None
    if not args.no_compare:  # the other precision on the same inputs
        other_prec = "mixed" if precision == "fp64" else "fp64"
        other = run_path(cs, prob, cfg, other_prec, args.steps, args.warmup, x0)
    del x0
    if args.calibrate_copy:  # a plain copy kernel of known size: reads and writes 1 GiB
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    lz = lanczos_figures(cs, prob, cfg, precision)
    fo = forces_figures(cs, prob, cfg, precision) if prob.n_atoms > 0 else None
    kp = kpoint_figures(cs, prob, cfg) if cfg.name in ("cfg1", "cfg2") else None
    cgbs = copy_gbs()
    kern = main_run["kernels"]
    # the dominant kernel among those with a roofline (the FP64 dense stage and copies have none)
    dominant = max(("hx_apply", "gram", "rotate"), key=lambda k: kern[k]["ms_per_step"])
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and precision == "fp64" and cfg.name == "cfg2":
        # counters of the same kernel source in the same launch configuration only
        # (one entry per tiling: autotune's pick among tilings that time within noise of
        # each other can differ from box to box)
        t = json.load(open(TRAFFIC_FILE))
        sc = main_run["stencil_choice"]
        if t.get("source_sha256_16") == kernel_source_hash("hx_apply.hip", "common.h"):
            for e in t.get("entries", []):
                if all(e["stencil_choice"].get(k) == sc[k]
                       for k in ("rows_per_thread", "row_groups", "projectors_in_stencil")):
                    traffic = e["bytes_per_launch"]
    g = main_run["gemm"]
    if dominant in ("gram", "rotate"):
        roof = {"bound": "mfma", "kernel": "gram+rotate", "achieved": g["executed_tflops"], "peak": g["peak_tflops"],
                "unit": "TFLOP/s", "frac": g["utilisation"], "traffic": None}
    else:
        hx_launches = m + 1
        roof = {"bound": "hbm", "kernel": "hx_apply", "achieved": main_run["hx_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": main_run["hx_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": main_run["hx_bytes_step"] / hx_launches,
                "avg_launch_ms": kern["hx_apply"]["avg_launch_ms"],
                # the whole H application: stencil pass plus the projector gather and scatter
                "with_nonlocal_gbs": main_run["hx_bytes_step"] / ((kern["hx_apply"]["ms_per_step"] +
                                                                  kern["nonlocal"]["ms_per_step"]) * 1e-3) / 1e9,
                "copy_gbs": cgbs, "frac_of_copy": main_run["hx_gbs"] / cgbs}

    out = {
        "metric": "CheFSI iter/s",
        "value": main_run["iter_per_s"],
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+bf16x3+f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {'x'.join(map(str, cfg.n))} grid h={cfg.h[0]} bohr, "
                               f"bc {''.join('PD'[b] for b in cfg.bc)}, FD order {cfg.fd_order}, "
                               f"{cfg.n_atoms} atoms x {cfg.nproj_per_atom} KB projectors, "
                               f"Ns={ns}, degree {m}, {precision}",
                   "grid": list(cfg.n), "ns": ns, "degree": m, "precision": precision, "nd": prob.nd},
        "roofline": roof,
        "hx_gbs": main_run["hx_gbs"],
        "gemm": g,
        "kernels": kern,
        "stencil_choice": main_run["stencil_choice"],
        "solve_ms": main_run["solve_ms"],
        "lanczos_lam_nd": lz,
        "nonlocal_forces": fo,
        "kpoint": kp,
    }
    if other is not None:
        out["compare"] = {
            "precision": other["precision"], "iter_per_s": other["iter_per_s"], "ms_per_step": other["ms_per_step"],
            "hx_gbs": other["hx_gbs"], "gemm": other["gemm"], "solve_ms": other["solve_ms"],
            "kernels": {k: round(v["ms_per_step"], 3) for k, v in other["kernels"].items()},
            "step_speedup_mixed_over_fp64": (other["iter_per_s"] / main_run["iter_per_s"] if precision == "fp64"
                                             else main_run["iter_per_s"] / other["iter_per_s"]),
        }
        if "refine_ms" in other:
            out["compare"]["refine_ms"] = other["refine_ms"]
    if "refine_ms" in main_run:
        out["refine_ms"] = main_run["refine_ms"]
    if not args.no_subrecords and cfg.name == "cfg2":
        # the configurations the mixed-precision target is about, outside the timed steps
        out["cfg3"] = workload_record(cs, "cfg3", steps=3, warmup=1, with_fp64=True)
        out["cfg4"] = workload_record(cs, "cfg4", steps=2, warmup=1, with_fp64=False)
        print(f"[bench] serving: {args.serving_requests} requests", file=sys.stderr, flush=True)
        out["cfg5_serving"] = serving_record(args, args.serving_requests)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cb = cpu_baseline(prob, cfg, args.cpu_columns)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                     "cfg1_whole_iter_per_s")}
        out["speedup_vs_cpu_oracle"] = out["value"] / cb["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
