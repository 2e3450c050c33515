#!/usr/bin/env python3
"""Throughput of the differential-BEM Levenberg-Marquardt step on one MI355X.

One step = one full LM iteration on a fresh batch of samples: mean colour,
forward sweep, residual and loss, gradient by the adjoint, J tiles and Gram
contraction for J^T J, float64 Cholesky solve, trial forward and
accept/reject (the whole hot path).  Default workload (--workload lm): 256
cubic handles x 32 segments (P = 5,120 parameters), 2,097,152 uniform samples
per step with Gaussian target noise sigma = 0.2, eps = 1e-2, 256 outer
elements per side.  --workload paper: the paper's own setting, 500 straight
handles (10 parameters each, one piece, Sobol placement at 1/20 width),
100,000 uniform samples per step, sigma = 0.1, targets clamped at 1.
Batches are generated and placed in HBM before the timed region.

Prints one JSON line.  `roofline` is for the kernel family with the largest
share of the timed region, from HIP events recorded by the library on its
launch stream; `cpu_baseline` times the FP64 CPU oracle on a bounded sample of
the same workload and extrapolates linearly.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sample×segment pairs/s and LM steps/s, FP32-mixed vs FP64 at 1e-4 color err"
PEAKS = {"fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12,
         "bf16_mfma": 2.5e15}
# Counters of the hot kernels (rocprofv3 --pmc passes over `bench.py --pmc-probe`: two 32,768-sample
# tiles of the LM workload, kernels serialised), each with the SHA-256 of the sources it was taken from
PMC_FILE = os.path.join(ROOT, "profiles", "lm_workload_counters.json")
CSRC = os.path.join(ROOT, "paper_2602_05492_amd", "csrc")
GRAM_TILE = 32768          # samples per split-BF16 Gram launch (the library's default tile)


def sources_sha(names) -> str:
    h = hashlib.sha256()
    for nm in names:
        h.update(open(os.path.join(CSRC, nm), "rb").read())
    return h.hexdigest()


def gram_tile_pairs(H: int, M: int, model: str) -> int:
    """256 x 256 output tiles the split-BF16 Gram computes: the upper triangle of the feature
    rows' tiles (three channel geometry blocks, each padded to 256 rows, then the shared colour
    and beta rows) without the pairs that lie in two different channels' geometry blocks."""
    G, C = (8, 4) if model == "cubic" else (4, 2)
    gp = -(-G * H // 256) * 256
    nt = -(-(3 * gp + C * H + M) // 256)

    def region(t):
        lo, hi = 256 * t, 256 * t + 255
        if lo >= 3 * gp:
            return -1
        if hi >= 3 * gp or lo // gp != hi // gp:
            return -2
        return lo // gp

    return sum(1 for i in range(nt) for j in range(i, nt)
               if not (region(i) >= 0 and region(j) >= 0 and region(i) != region(j)))


def pmc_record():
    try:
        return json.load(open(PMC_FILE))
    except (OSError, ValueError):
        return None


# algorithmic work per unit (float32 flops, FMA = 2)
F_HANDLE_PAIR = 110.0      # forward: one sample x one handle segment
F_BOUNDARY_PAIR = 40.0     # forward / adjoint: one sample x one outer element
F_GRAD_PAIR = 300.0        # adjoint or J-tile: one sample x one handle segment


WORKLOADS = {"lm": 5, "paper": 6, "medium": 2}
WORKLOAD_TEXT = {
    "medium": "medium: 32 crossing cubic handles x 16 segments (P = 640), 262,144 uniform samples per step, "
              "sigma 0.2, eps 1e-2, 1,024 outer elements",
    "lm": "LM normal equations: 256 cubic handles x 32 segments (P = 5,120), 2,097,152 uniform samples per step, "
          "sigma 0.2, eps 1e-2, 1,024 outer elements",
    "paper": "paper-native: 500 straight handles x 1 segment (P = 5,000; Sobol placement, length 1/20), 100,000 "
             "uniform samples per step, sigma 0.1, targets clamped at 1, eps 1e-2, 1,024 outer elements",
}
# feature rows per handle of the normal equations: geometry per channel, channel-shared colour
FEATURE_ROWS = {"cubic": (8, 4), "straight": (4, 2)}


def make_context(wl, tile_rows: int = 0):
    from paper_2602_05492_amd import bem as B
    return B.Context(segs_per_handle=wl.S, eps=wl.eps, elems_per_side=wl.elems_per_side, handle_model=wl.spec.model,
                     tile_rows=tile_rows)


def make_target(ctx, wl, tht, x, step):
    """Noise-free reconstruction of the ground truth plus the workload's noise (clamped where the
    workload clamps), on the GPU."""
    import torch
    T = ctx.eval(tht, x, wl.cbar_true, "fp64") + wl.spec.sigma * torch.from_numpy(wl.noise(step)).cuda()
    return T.clamp_(max=wl.spec.target_max) if wl.spec.target_max is not None else T


def gram_entries(H: int, M: int, model: str = "cubic") -> int:
    """Distinct Gram entries J^T J needs per sample (symmetric blocks counted once)."""
    fg, fc = FEATURE_ROWS[model]
    g, s = fg * H, fc * H + M
    return 3 * (g * (g + 1) // 2) + 3 * g * s + s * (s + 1) // 2


def counters(kernel: str):
    """The committed counter record of a kernel, or None when there is none or its sources have
    changed since it was taken."""
    rec = pmc_record()
    k = rec.get("kernels", {}).get(kernel) if rec else None
    if not k or k.get("source_sha256") != sources_sha(k.get("source_files", [])):
        return None
    return k


def gram_alg_bytes(H: int, M: int, model: str) -> float:
    """Algorithmic HBM bytes of one split-BF16 Gram launch: the feature tile read once (hi and lo
    planes, W rows x the tile's samples) and the partial-Gram tiles of its work list read and
    written once (8-byte entries, 3 parts)."""
    fg, fc = FEATURE_ROWS[model]
    W = 3 * (-(-fg * H // 256) * 256) + fc * H + M
    return W * GRAM_TILE * 4.0 + 2 * 3 * gram_tile_pairs(H, M, model) * 256 * 256 * 8.0


def gram_traffic(samples_per_launch: int):
    """HBM bytes per Gram launch from the committed counter run (FETCH_SIZE and WRITE_SIZE scaled by
    what they read for a plain copy), or None."""
    g = counters("k_gram_bf16x3_lds")
    if not g or samples_per_launch != GRAM_TILE:
        return None
    return g["hbm_bytes"]


def valu_fraction(kernel: str, pairs_per_s_in_step):
    """float32 VALU rate of a sweep-type kernel: the counter flops per pair (FMA = 2) times its pair
    rate, in the timed step (shared with other kernels) and alone (the counter run), against the
    float32 vector peak (packed) and the non-packed FMA ceiling (half of it)."""
    k = counters(kernel)
    if not k or "fp32_flops_per_pair" not in k:
        return None
    fpp = k["fp32_flops_per_pair"]
    out = {"kernel": kernel, "fp32_flops_per_pair": fpp, "valu_insts_per_pair": k["valu_insts_per_pair"],
           "compiler": k.get("compiler"),
           "alone": {"pairs_per_s": k["pairs_per_s_alone"], "tflops": k["tflops_alone"],
                     "frac": k["tflops_alone"] / (PEAKS["fp32_vector"] / 1e12),
                     "frac_of_unpacked_peak": k["tflops_alone"] / (PEAKS["fp32_vector"] / 2e12),
                     "clock_ghz": k["clock_ghz"]}}
    if pairs_per_s_in_step:
        tf = fpp * pairs_per_s_in_step / 1e12
        out["in_step"] = {"pairs_per_s": pairs_per_s_in_step, "tflops": tf, "frac": tf / (PEAKS["fp32_vector"] / 1e12),
                          "frac_of_unpacked_peak": tf / (PEAKS["fp32_vector"] / 2e12)}
    return out


def pmc_probe() -> int:
    """Small run for counters: one mixed split-BF16 LM step of the LM workload on batch 0 (its forward
    sweeps on the cell-ordered samples, its 64 J tiles of 32,768 samples and their Gram launches,
    exactly as in the timed step), one mixed adjoint of the adjoint workload (4,194,304 samples, as
    `--workload adjoint` times it; the cotangent's values do not change the work), then a plain
    256 MiB device copy whose counters calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2602_05492_amd import bem as B
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(5)
    ctx = make_context(wl)
    tht = torch.from_numpy(wl.theta_true).cuda()
    xs = torch.from_numpy(wl.samples(0)).cuda()
    T = make_target(ctx, wl, tht, xs, 0)
    th = torch.from_numpy(wl.theta0).cuda()
    st = B.new_lm_state(wl.lam0, 0)
    ctx.lm_step(th, xs, T, st, "bf16x3_mfma", "mixed")
    wa = W.make_config(4)
    xa = torch.from_numpy(wa.samples(0)).cuda()
    ra = (1e-6 * torch.from_numpy(wa.noise(0))).float().cuda()
    make_context(wa).vjp(torch.from_numpy(wa.theta0).cuda(), xa, ra, "mixed")
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("pmc probe done", flush=True)
    return 0


def power_probe(seconds: float = 6.0) -> int:
    """Board power and shader clock (read-only sysfs: hwmon power1_input, pp_dpm_sclk), sampled every
    20 ms while the LM workload's mixed forward sweep runs back to back, then while its normal
    equations (J tiles and split-BF16 Gram on two streams, bem_jtj) run back to back; one JSON line
    with the median, 10th and 90th percentiles per phase."""
    import glob
    import re
    import threading
    import torch
    from paper_2602_05492_amd import bem as B
    from paper_2602_05492_amd import workload as W
    dev = sorted(glob.glob("/sys/class/drm/card*/device"))
    pw = [p for d in dev for p in glob.glob(d + "/hwmon/hwmon*/power1_input")]
    sc = [d + "/pp_dpm_sclk" for d in dev if os.path.exists(d + "/pp_dpm_sclk")]

    def power_w():
        try:
            with open(pw[0]) as f:
                return int(f.read()) / 1e6
        except (OSError, ValueError, IndexError):
            return None

    def sclk_mhz():
        try:
            with open(sc[0]) as f:
                m = re.search(r"(\d+)Mhz \*", f.read())
            return int(m.group(1)) if m else None
        except (OSError, IndexError):
            return None

    wl = W.make_config(5)
    ctx = make_context(wl)
    th = torch.from_numpy(wl.theta0).cuda()
    x = torch.from_numpy(wl.samples(0)).cuda()
    r = (wl.spec.sigma * torch.from_numpy(wl.noise(0))).float().cuda()
    phases = {"forward_sweep": lambda: ctx.eval(th, x, wl.cbar_true, "mixed"),
              "normal_equations": lambda: ctx.jtj(th, x, r, "bf16x3_mfma", "mixed")}
    for f in phases.values():
        f()
    torch.cuda.synchronize()
    label, stop, samples = ["idle"], [False], []

    def sampler():
        while not stop[0]:
            samples.append((label[0], power_w(), sclk_mhz()))
            time.sleep(0.02)

    t = threading.Thread(target=sampler, daemon=True)
    t.start()
    calls = {}
    for name, f in phases.items():
        time.sleep(0.5)
        label[0] = name
        t0, n = time.perf_counter(), 0
        while time.perf_counter() - t0 < seconds:
            f()
            n += 1
            if n % 4 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        calls[name] = {"calls": n, "ms_per_call": (time.perf_counter() - t0) * 1e3 / n}
        label[0] = "idle"
    stop[0] = True
    t.join()

    def stats(v):
        v = sorted(x for x in v if x is not None)
        return {"n": len(v), "median": v[len(v) // 2], "p10": v[len(v) // 10], "p90": v[9 * len(v) // 10]} if v else None

    out = {"what": "board power (W) and shader clock (MHz) per phase, LM workload", "sources": pw[:1] + sc[:1]}
    for name in phases:
        out[name] = {"power_w": stats([p for l, p, c in samples if l == name]),
                     "sclk_mhz": stats([c for l, p, c in samples if l == name]), **calls[name]}
    print(json.dumps(out), flush=True)
    return 0


def lm_curve(steps: int, gram: str, prec: str, workload: str, compat: int, ref: bool = False) -> int:
    """LM iterations of a workload with fresh samples per step; one JSON line per step.  With ref,
    each step's direction is also compared with the plain float64 step (float64 sweeps and Gram)
    taken from the same parameters, damping and batch."""
    import numpy as np
    import torch
    from paper_2602_05492_amd import bem as B
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(WORKLOADS[workload])
    ctx = make_context(wl)
    tht = torch.from_numpy(wl.theta_true).cuda()
    c = (np.arange(512) + 0.5) / 512
    grid = torch.from_numpy(np.stack(np.meshgrid(c, c, indexing="xy"), -1).reshape(-1, 2).copy()).cuda()
    truth = ctx.eval(tht, grid, wl.cbar_true, "fp64")
    theta = torch.from_numpy(wl.theta0).cuda()
    st = B.new_lm_state(wl.lam0, 0, compat=compat)

    def rmse(cbar):
        u = ctx.eval(theta, grid, tuple(cbar), "fp64")
        return float(torch.sqrt(((u - truth) ** 2).mean()))

    for i in range(steps):
        x = torch.from_numpy(wl.samples(i)).cuda()
        T = make_target(ctx, wl, tht, x, i)
        if i == 0:   # the start, with the mean colour the first step will use
            print(json.dumps({"step": 0, "rmse": rmse(T.mean(0).tolist())}), flush=True)
        dir_err = None
        if ref:
            th64 = theta.clone()
            st64 = B.new_lm_state(st.lam, 0, compat=compat)
            st64.cbar_sum[:] = st.cbar_sum[:]
            st64.cbar_count = st.cbar_count
            ctx.lm_step(th64, x, T, st64, "fp64", "fp64")
        th_before = theta.clone()
        t = time.perf_counter()
        ctx.lm_step(theta, x, T, st, gram, prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        if ref and st.accepted and st64.accepted:
            d, d64 = (theta - th_before).flatten(), (th64 - th_before).flatten()
            dir_err = float(torch.linalg.vector_norm(d - d64) / torch.linalg.vector_norm(d64))
        rec = {"step": i + 1, "loss_before": st.loss_before, "loss_after": st.loss_after,
               "accepted": int(st.accepted), "lambda": st.lam, "ms": ms, "rmse": rmse(st.cbar)}
        if ref:
            rec["fp64_accepted"] = int(st64.accepted)
            rec["step_dir_rel_err_vs_fp64"] = dir_err
        print(json.dumps(rec), flush=True)
    return 0


# ---- CPU baseline: the FP64 oracle on the host's cores ----------------------------------------
# Worker processes are started (spawn) before this process touches the GPU; each runs the oracle
# single-threaded on its own chunk of the same workload, so the per-sample times below are
# measured with every worker busy.  The one-time boundary factor is not part of a step.
def _cpu_worker_init():
    import numpy  # noqa: F401  (load BLAS before limiting its threads)
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits
    global _CPU_LIMIT
    _CPU_LIMIT = threadpool_limits(limits=1)


def _cpu_chunk(job):
    """(kind, config, lo, hi) -> seconds the oracle takes for that piece on one core."""
    import numpy as np
    import oracle as O
    from paper_2602_05492_amd import workload as W
    kind, config, lo, hi = job
    wl = W.make_config(config)
    S, eps = wl.S, wl.eps
    th = wl.theta0 if wl.spec.model == "cubic" else O.straight.embed(wl.theta0)
    bnd = O.boundary(wl.elems_per_side)
    if kind in ("rhs", "dF"):
        pts = bnd.gp.reshape(-1, 2)[lo:hi]
        t = time.perf_counter()
        if kind == "rhs":
            O.handle_term(pts, th, S, eps)
        else:
            O.handle_term_jacobian(pts, th, S, eps)
        return time.perf_counter() - t
    x = wl.samples(0, n=max(hi, 1))[lo:hi]
    t = time.perf_counter()
    if kind == "forward":
        O.handle_term(x, th, S, eps)
        O.element_weights(x, bnd)
    else:                                    # J rows (Z given) and their Gram update
        Z = np.zeros((bnd.M, 3, th.size))
        J = O.handle_term_jacobian(x, th, S, eps) + np.einsum("nj,jcp->ncp", O.element_weights(x, bnd), Z)
        Jr = J.reshape(-1, th.size)
        _ = Jr.T @ Jr
    return time.perf_counter() - t


def cpu_cores() -> int:
    """Host cores the baseline uses: every core this process may run on, at most 16 (the host
    share of one GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(config: int) -> dict:
    """The FP64 oracle timed on bounded pieces of one LM step of the workload, on all host
    cores, extrapolated linearly in the sample count to one step."""
    import multiprocessing as mp

    import numpy as np
    from scipy.linalg import cho_factor
    from threadpoolctl import threadpool_limits

    import oracle as O
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(config)
    C = cpu_cores()
    n_fwd, n_jac, n_gp = 256, 32, 48        # samples and boundary Gauss points per worker
    bnd = O.boundary(wl.elems_per_side)      # one-time factor (SVD), outside the timed pieces
    ng = bnd.gp.reshape(-1, 2).shape[0]
    P = wl.P
    with mp.get_context("spawn").Pool(C, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_chunk, [("forward", config, i, i + 1) for i in range(C)])          # warm the workers

        def timed(jobs):
            t = time.perf_counter()
            pool.map(_cpu_chunk, jobs)
            return time.perf_counter() - t

        t_fwd = timed([("forward", config, i * n_fwd, (i + 1) * n_fwd) for i in range(C)]) / (C * n_fwd)
        t_jac = timed([("jac", config, i * n_jac, (i + 1) * n_jac) for i in range(C)]) / (C * n_jac)
        # the boundary right-hand side and dF/dtheta on n_gp Gauss points per worker, scaled to all ng
        t_rhs = timed([("rhs", config, i * n_gp, (i + 1) * n_gp) for i in range(C)]) * ng / (C * n_gp)
        t_dF = timed([("dF", config, i * n_gp, (i + 1) * n_gp) for i in range(C)]) * ng / (C * n_gp)
    th = wl.theta0 if wl.spec.model == "cubic" else O.straight.embed(wl.theta0)
    rng = np.random.default_rng(0)
    with threadpool_limits(limits=C):
        dF = rng.standard_normal((bnd.M, 3 * th.size))
        t = time.perf_counter()
        _ = bnd.Apinv @ dF                   # Z = A+ dF/dtheta (boundary_derivative_values)
        t_z = time.perf_counter() - t
        B = rng.standard_normal((P, P // 4))
        Hd = B @ B.T + P * np.eye(P)
        t = time.perf_counter()
        cho_factor(Hd, lower=True)           # damped_step's Cholesky of the P x P system
        t_chol = time.perf_counter() - t
    N = wl.N
    step = 2 * (N * t_fwd + t_rhs) + t_dF + t_z + N * t_jac + t_chol
    return {"value": 1.0 / step, "unit": "LM steps/s", "cores": C, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"oracle (numpy FP64) on {C} host cores ({cpu_model()}), {C} single-threaded worker processes: "
                       f"forward on {C * n_fwd} samples, J rows + Gram update on {C * n_jac} samples, the boundary "
                       f"right-hand side and dF/dtheta at {C * n_gp} of the {ng} Gauss points, then with {C} BLAS threads "
                       f"Z = A+ dF/dtheta ({bnd.M} x {bnd.M} by {bnd.M} x {3 * th.size}) and the Cholesky of a "
                       f"{P} x {P} system; extrapolated linearly to one step of {N:,} samples (2 forwards, "
                       f"2 right-hand sides, dF/dtheta, Z, J^T J, Cholesky): {step:.3e} s/step "
                       f"(per sample: forward {t_fwd * C:.3e} s, J rows + Gram {t_jac * C:.3e} s on one core).")}


def forward_mode(steps: int, warmup: int, do_cpu: bool) -> int:
    """Near-singular forward (128 cubic handles x 32 segments, 1,048,576 samples of which 10% lie
    within 1e-3 of a segment): mixed bem_eval throughput, its float64 near-pair share, and the
    colour error against the float64 GPU path (validated against the oracle by the GPU tests),
    split into the near and the uniform samples."""
    config = 3
    cpu = cpu_forward_baseline(config) if do_cpu else None
    import torch
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(config)
    ctx = make_context(wl)
    N, K, M = wl.N, wl.H * wl.S, ctx.M
    th = torch.from_numpy(wl.theta_true).cuda()
    x = torch.from_numpy(wl.samples(0)).cuda()
    for _ in range(warmup):
        ctx.eval(th, x, wl.cbar_true, "mixed")
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        u = ctx.eval(th, x, wl.cbar_true, "mixed")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    t0 = time.perf_counter()
    u64 = ctx.eval(th, x, wl.cbar_true, "fp64")
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3
    err = (u.double() - u64).abs().amax(dim=1)
    n_near = int(round(wl.spec.near_frac * N))
    pairs = N * (K + M)
    out = {"metric": "sample x segment pairs/s (mixed forward, near-singular samples)", "value": pairs / (ms * 1e-3),
           "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": W.SPECS[config].name, "handles": wl.H, "segs_per_handle": wl.S, "samples": N,
                      "outer_elements": M, "near_samples": n_near},
           "fp64_gpu_ms": ms64, "fp64_pairs_per_s": pairs / (ms64 * 1e-3), "speedup_vs_fp64_gpu": ms64 / ms,
           "color_err_vs_fp64": {"max_abs_all": float(err.max()), "max_abs_uniform": float(err[: N - n_near].max()),
                                 "max_abs_near": float(err[N - n_near:].max()) if n_near else None, "bar": 1e-4},
           "kernel_ms_per_eval": {k: v[0] / steps for k, v in prof.items() if v[1] > 0},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


def adjoint_mode(steps: int, warmup: int, do_cpu: bool) -> int:
    """Differentiation workload (256 cubic handles x 32 segments, 4,194,304 samples): bem_vjp
    throughput of the mean-squared-error gradient, mixed and float64, and the gradient's error."""
    config = 4
    cpu = cpu_adjoint_baseline(config) if do_cpu else None
    import torch
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(config)
    ctx = make_context(wl)
    N, K, M = wl.N, wl.H * wl.S, ctx.M
    tht = torch.from_numpy(wl.theta_true).cuda()
    th = torch.from_numpy(wl.theta0).cuda()
    x = torch.from_numpy(wl.samples(0)).cuda()
    T = make_target(ctx, wl, tht, x, 0)
    g64 = (2.0 / (3 * N)) * (ctx.eval(th, x, wl.cbar_true, "fp64") - T)       # d(mean squared error)/du
    g32 = g64.float()
    for _ in range(warmup):
        ctx.vjp(th, x, g32, "mixed")
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        gm = ctx.vjp(th, x, g32, "mixed")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.vjp(th, x, g64, "fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gd = ctx.vjp(th, x, g64, "fp64")
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3
    rel = float((gm - gd).abs().max() / gd.abs().max())
    pairs = N * (K + M)
    seg_ms = prof["vjp_segments"][0] / steps if prof["vjp_segments"][1] else None
    vjp_valu = valu_fraction("k_vjp_segments", N * K / (seg_ms * 1e-3) if seg_ms else None)
    out = {"metric": "sample x segment pairs/s (mixed adjoint, bem_vjp)", "value": pairs / (ms * 1e-3),
           "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": W.SPECS[config].name, "handles": wl.H, "segs_per_handle": wl.S, "samples": N,
                      "params": wl.P, "outer_elements": M},
           "handle_pairs_per_s": N * K / (ms * 1e-3), "fp64_gpu_ms": ms64, "fp64_pairs_per_s": pairs / (ms64 * 1e-3),
           "speedup_vs_fp64_gpu": ms64 / ms,
           "grad_rel_err_vs_fp64": {"max_abs_over_max": rel, "bar": 1e-3}, "vjp_valu": vjp_valu,
           "kernel_ms_per_vjp": {k: v[0] / steps for k, v in prof.items() if v[1] > 0},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


def cpu_forward_baseline(config: int) -> dict:
    import multiprocessing as mp
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(config)
    C, n = cpu_cores(), 256
    with mp.get_context("spawn").Pool(C, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_chunk, [("forward", config, i, i + 1) for i in range(C)])
        t = time.perf_counter()
        pool.map(_cpu_chunk, [("forward", config, i * n, (i + 1) * n) for i in range(C)])
        t = (time.perf_counter() - t) / (C * n)
    K, M = wl.H * wl.S, 4 * wl.elems_per_side
    return {"value": (K + M) / t, "unit": "pairs/s", "cores": C, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"oracle (numpy FP64) forward on {C * n} samples of the workload, {C} single-threaded worker "
                      f"processes on {C} host cores ({cpu_model()}); the boundary solve (per evaluation, "
                      f"independent of N) is not included."}


def cpu_adjoint_baseline(config: int) -> dict:
    import multiprocessing as mp
    from paper_2602_05492_amd import workload as W
    wl = W.make_config(config)
    C, n = cpu_cores(), 16
    with mp.get_context("spawn").Pool(C, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_chunk, [("forward", config, i, i + 1) for i in range(C)])
        t = time.perf_counter()
        pool.map(_cpu_chunk, [("jac", config, i * n, (i + 1) * n) for i in range(C)])
        t = (time.perf_counter() - t) / (C * n)
    K, M = wl.H * wl.S, 4 * wl.elems_per_side
    return {"value": (K + M) / t, "unit": "pairs/s", "cores": C, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"oracle (numpy FP64) gradient by explicit Jacobian rows on {C * n} samples of the workload "
                      f"(the oracle's vjp forms J), {C} single-threaded worker processes on {C} host cores "
                      f"({cpu_model()})."}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--gram", default="bf16x3_mfma", choices=["fp64", "fp32_mfma", "bf16x3_mfma", "fp64_valu"])
    ap.add_argument("--fp64-ref", type=int, default=1,
                    help="also time the plain FP64 GPU step (one warm-up, median of 3) for the speedup")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="samples per J tile of the normal equations (0: the library's choice)")
    ap.add_argument("--compat", type=int, default=0,
                    help="enforce the compatibility condition in every LM step (constrained step + re-projection)")
    ap.add_argument("--workload", default="lm", choices=sorted(WORKLOADS) + ["near", "adjoint"],
                    help="lm: 256 cubic handles x 32 segments, 2,097,152 samples (LM steps/s); paper: 500 straight "
                         "handles, 100,000 samples (LM steps/s); medium: 32 crossing cubic handles x 16 segments, "
                         "262,144 samples (LM steps/s; --prec fp64 --gram fp64 for the plain FP64 path); near: mixed forward with near-singular samples, "
                         "1,048,576 samples (pairs/s); adjoint: bem_vjp at 4,194,304 samples (pairs/s)")
    ap.add_argument("--pmc-probe", action="store_true", help="only the small run profiled for byte counters")
    ap.add_argument("--power-probe", action="store_true",
                    help="only sample board power and shader clock during the forward sweep and the normal equations")
    ap.add_argument("--lm-curve-ref", action="store_true",
                    help="with --lm-curve: also take the float64 step from the same state each step and report the "
                         "step direction's relative error")
    ap.add_argument("--lm-curve", type=int, default=0,
                    help="instead of timing: run this many LM steps (fresh samples each) and print loss, lambda and "
                         "RMSE against the noise-free truth on the 512 x 512 pixel-centre grid per step")
    args = ap.parse_args()
    if args.pmc_probe:
        return pmc_probe()
    if args.power_probe:
        return power_probe()
    if args.lm_curve:
        return lm_curve(args.lm_curve, args.gram, args.prec, args.workload, args.compat, args.lm_curve_ref)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the sample-sharded multi-GPU path is not built; "
              "run with --gpus 1", file=sys.stderr)
        return 2
    if args.workload == "near":
        return forward_mode(args.steps, args.warmup, bool(args.cpu_baseline))
    if args.workload == "adjoint":
        return adjoint_mode(args.steps, args.warmup, bool(args.cpu_baseline))

    # the CPU baseline's worker processes run before this process initialises the GPU
    cpu = cpu_baseline(WORKLOADS[args.workload]) if args.cpu_baseline else None
    if cpu:
        print(f"cpu baseline: {cpu['value']:.3e} LM steps/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import numpy as np
    import torch
    from paper_2602_05492_amd import bem as B
    from paper_2602_05492_amd import workload as W

    wl = W.make_config(WORKLOADS[args.workload])
    ctx = make_context(wl, args.tile_rows)
    H, S, N, M = wl.H, wl.S, wl.N, ctx.M
    K = H * S
    nb = args.warmup + args.steps
    tht = torch.from_numpy(wl.theta_true).cuda()
    batches = []
    for i in range(nb):
        x = torch.from_numpy(wl.samples(i)).cuda()
        batches.append((x, make_target(ctx, wl, tht, x, i)))
    theta = torch.from_numpy(wl.theta0).cuda()
    st = B.new_lm_state(wl.lam0, 0, compat=args.compat)
    for i in range(args.warmup):
        ctx.lm_step(theta, batches[i][0], batches[i][1], st, args.gram, args.prec)
        print(f"warmup {i}: loss {st.loss_before:.6e} -> {st.loss_after:.6e} accepted {st.accepted}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile(True)
    losses = []
    t0 = time.perf_counter()
    for i in range(args.warmup, nb):
        ctx.lm_step(theta, batches[i][0], batches[i][1], st, args.gram, args.prec)
        losses.append((st.loss_before, st.loss_after, int(st.accepted)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    for i, l in enumerate(losses):
        print(f"step {i}: loss {l[0]:.6e} -> {l[1]:.6e} accepted {l[2]}", file=sys.stderr, flush=True)
    ms = (t1 - t0) * 1e3 / args.steps
    value = 1e3 / ms

    # algorithmic work of each kernel family in the timed region
    steps = args.steps
    work = {
        "sweep_mixed": prof["sweep_mixed"][1] * (F_HANDLE_PAIR * N * K + F_BOUNDARY_PAIR * N * M),
        "sweep_f64": prof["sweep_f64"][1] * (F_HANDLE_PAIR * N * K + F_BOUNDARY_PAIR * N * M),
        "vjp_segments": steps * F_GRAD_PAIR * (N + 3 * M) * K,
        "vjp_elements": steps * F_BOUNDARY_PAIR * N * M,
        "features": steps * F_GRAD_PAIR * (N + 3 * M) * K,
        "gram_mfma": steps * 2.0 * N * gram_entries(H, M, wl.spec.model),
        "gram_f64": steps * 2.0 * N * gram_entries(H, M, wl.spec.model),
    }
    peak_of = {"sweep_mixed": ("alu", PEAKS["fp32_vector"]), "sweep_f64": ("alu", PEAKS["fp64_vector"]),
               "vjp_segments": ("alu", PEAKS["fp32_vector"] if args.prec == "mixed" else PEAKS["fp64_vector"]),
               "vjp_elements": ("alu", PEAKS["fp32_vector"]),
               "features": ("alu", PEAKS["fp32_vector"] if args.prec == "mixed" else PEAKS["fp64_vector"]),
               "gram_mfma": ("mfma", PEAKS["bf16_mfma"] if args.gram == "bf16x3_mfma" else PEAKS["fp32_mfma"]),
               "gram_f64": ("mfma", PEAKS["fp64_mfma"]) if args.gram == "fp64" else ("alu", PEAKS["fp64_vector"])}
    timed = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max((k for k in timed if k in work), key=lambda k: timed[k][0])
    tot_ms, launches = timed[dom]
    achieved = work[dom] / (tot_ms * 1e-3) / 1e12
    bound, peak = peak_of[dom]
    # the committed byte counters were taken on the LM workload's Gram
    traffic = (gram_traffic(GRAM_TILE) if (dom == "gram_mfma" and args.gram == "bf16x3_mfma" and args.workload == "lm"
                                           and args.tile_rows in (0, GRAM_TILE)) else None)
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / (peak / 1e12), "traffic": traffic, "launches": launches,
                "avg_launch_ms": tot_ms / launches}
    if traffic is not None:
        # context from the same counter run: the clock under the Gram launch alone (GRBM_GUI_ACTIVE
        # per XCD over its duration) and the MFMA work it issues (3 products per entry) against
        # the dense bf16 peak at that clock
        g = counters("k_gram_bf16x3_lds")
        issued = gram_tile_pairs(H, M, wl.spec.model) * 256 * 256 * 2.0 * GRAM_TILE * 3
        roofline["alone"] = {"ms": g["duration_ms"], "clock_ghz": g["clock_ghz"],
                             "mfma_issued_pflops": issued / (g["duration_ms"] * 1e-3) / 1e15,
                             "frac_of_peak_at_clock": issued / (g["duration_ms"] * 1e-3) / (2.5e15 * g["clock_ghz"] / 2.4),
                             "algorithmic_bytes": (gram_alg_bytes(H, M, wl.spec.model)
                                                   if wl.spec.model == "cubic" else None)}
    fwd_ms = prof["sweep_mixed" if args.prec == "mixed" else "sweep_f64"]
    pairs_fwd = (N * (K + M)) / (fwd_ms[0] / fwd_ms[1] * 1e-3) if fwd_ms[1] else None
    vjp_ms = prof["vjp_segments"][0] + prof["vjp_elements"][0]
    pairs_vjp = steps * (N * (K + M)) / (vjp_ms * 1e-3) if vjp_ms > 0 else None
    feat_ms = prof["features"][0]
    pairs_feat = steps * N * K / (feat_ms * 1e-3) if feat_ms > 0 else None

    # the VALU kernels against the float32 vector peak (packed FP32 counts twice; without it the
    # vector ceiling is half of that), from the committed counters of the LM workload
    lm_mixed = args.prec == "mixed" and args.workload == "lm"
    sweep_valu = valu_fraction("k_sweep_far", pairs_fwd) if lm_mixed else None
    if sweep_valu:
        sw = counters("k_sweep_far")
        samples_per_s = pairs_fwd / (K + M)
        sweep_valu["transcendental_frac"] = sw["trans_per_pair"] * pairs_fwd / (PEAKS["fp32_vector"] / 16)
        sweep_valu["hbm_gbps"] = sw["hbm_bytes"] / 65536 * samples_per_s / 1e9
    features_valu = valu_fraction("k_features_far", pairs_feat) if lm_mixed else None

    # colour error of the mixed forward against the float64 path at the start parameters, over
    # every sample of the first batch (the metric's "at 1e-4 color err")
    x0 = batches[0][0]
    th0 = torch.from_numpy(wl.theta0).cuda()
    cbar0 = tuple(float(v) for v in batches[0][1].mean(0))
    u_mixed = ctx.eval(th0, x0, cbar0, "mixed")
    u_f64 = ctx.eval(th0, x0, cbar0, "fp64")
    color_err = {"max_abs": float((u_mixed.double() - u_f64).abs().max()), "samples": N, "bar": 1e-4,
                 "against": "float64 GPU path (oracle-validated) at the start parameters, every sample of batch 0"}
    del u_mixed, u_f64

    speedup = None
    fp64 = None
    step_err = None
    if args.fp64_ref and args.prec == "mixed":
        # the plain float64 GPU step (float64 sweeps, float64 Gram on float64 MFMA): one warm-up,
        # then the median of 3, each from the start parameters on batch 0
        times, gram_ms = [], []
        for rep in range(4):
            th64 = torch.from_numpy(wl.theta0).cuda()
            st64 = B.new_lm_state(wl.lam0, 0, compat=args.compat)
            torch.cuda.synchronize()
            ctx.profile(rep > 0)
            t = time.perf_counter()
            ctx.lm_step(th64, batches[0][0], batches[0][1], st64, "fp64", "fp64")
            torch.cuda.synchronize()
            if rep > 0:
                times.append((time.perf_counter() - t) * 1e3)
                gram_ms.append(ctx.profile_read()["gram_f64"][0])
            ctx.profile(False)
        fp64_ms = float(np.median(times))
        g_ms = float(np.median(gram_ms))
        fp64 = {"ms_per_step": fp64_ms, "runs_ms": times, "gram": "fp64 (float64 MFMA)",
                "gram_ms": g_ms, "gram_tflops": 2.0 * N * gram_entries(H, M, wl.spec.model) / (g_ms * 1e-3) / 1e12,
                "gram_peak_tflops": PEAKS["fp64_mfma"] / 1e12}
        speedup = fp64_ms / ms
        print(f"fp64 reference step: {fp64_ms:.1f} ms (median of {times}), Gram {g_ms:.1f} ms", file=sys.stderr,
              flush=True)
        # step direction of the reduced-precision Grams against the FP64 step (same batch, same start)
        step_err = {}
        d64 = (th64 - torch.from_numpy(wl.theta0).cuda()).flatten()
        for gm in ["bf16x3_mfma", "fp32_mfma"]:
            thg = torch.from_numpy(wl.theta0).cuda()
            stg = B.new_lm_state(wl.lam0, 0, compat=args.compat)
            ctx.lm_step(thg, batches[0][0], batches[0][1], stg, gm, "mixed")
            dg = (thg - torch.from_numpy(wl.theta0).cuda()).flatten()
            step_err[gm] = (float(torch.linalg.vector_norm(dg - d64) / torch.linalg.vector_norm(d64))
                            if (st64.accepted and stg.accepted) else None)
        print(f"step direction vs fp64: {step_err}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "LM steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "handle_model": wl.spec.model,
                   "handles": H, "segs_per_handle": S, "samples": N, "params": wl.P, "outer_elements": M,
                   "prec": args.prec, "gram": args.gram, "compat": args.compat, "parallelism": "single GPU"},
        "pairs_per_s_forward": pairs_fwd, "pairs_per_s_adjoint": pairs_vjp, "color_err_vs_fp64": color_err,
        "fp64_gpu": fp64, "speedup_vs_fp64_gpu": speedup,
        "step_direction_rel_err_vs_fp64": step_err,
        "kernel_ms_per_step": {k: v[0] / steps for k, v in timed.items()},
        "sweep_valu": sweep_valu, "features_valu": features_valu, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
