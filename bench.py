#!/usr/bin/env python3
"""Benchmark of the space-time SU solver hot path on one MI355X.

One step = one full outer (Newton) iteration of the space-time solver from a
fixed state u^1 (the iterate after one FP64 Newton step from the lifted
initial datum): w-update, linearization (theta on the Greville grid, truncated
SVDs of theta and of the reaction coefficient), residual N(u^1) with the exact
ionic current at the Gauss points, FGMRES(30) with the fast-diagonalization
preconditioner to an FP64 true relative residual of 1e-8 (mixed precision:
FP32 or BF16 operator/preconditioner inside FP64 iterative refinement), and
the Newton update.  Every step solves the identical system, so FP64 and mixed
runs are comparable.  Inputs are resident in HBM before the timed region.

Prints one JSON line (see the fields below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # bytes/s, MI355X HBM3E
PEAK_FP64 = 78.6e12        # flop/s, FP64 vector and dense MFMA
PEAK_FP32 = 157.3e12       # flop/s, FP32 dense MFMA (and the published FP32 vector figure)
# FP32 vector arithmetic without packed FP32 instructions (the kernels are
# built without them): 256 CUs x 64 lanes x 2 flop per FMA x 2.4 GHz
PEAK_FP32_VALU = 256 * 64 * 2 * 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=[0, 1, 2, 4])
    ap.add_argument("--prec", default="mixed_fp32", choices=["fp64", "mixed_fp32", "mixed_bf16"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra workloads (config 2 in BF16, config 4 mixed FP32) of the default line")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precond", type=int, default=0, choices=[0, 1],
                    help="0: fast diagonalization (Sec. 3.2); 1: banded time solve per spatial mode")
    ap.add_argument("--max-rank", type=int, default=None,
                    help="cap of each low rank (default 48; 16 for config 4 to fit HBM)")
    ap.add_argument("--serve", action="store_true", help="run only the serving stream (512 requests)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream sampled in the default run (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=6)
    ap.add_argument("--compare-su", action="store_true",
                    help="fixed-point scheme of Section 3.1 (exact C_r, alpha = 0.5, stop at 1e-4) with and "
                         "without the SU term on config 1: iteration counts and times")
    ap.add_argument("--kernel-probe", type=int, default=0, metavar="REPS",
                    help="run only the hardware-counter probe (1 GiB copy, then REPS operator applications)")
    return ap.parse_args()


def serving(n_requests, slots):
    """Config 3: seeded stream of 2D solves, Poisson arrivals at 20 req/s,
    mixed FP32, linear and nonlinear tolerance 1e-8, continuous batching,
    banded time preconditioner."""
    import st_workloads as W
    from paper_2311_17500_amd.binding import MIXED_FP32
    from paper_2311_17500_amd.serve import Server, summarize
    reqs = W.serve_stream(512, 0)[:n_requests]
    # banded time preconditioner: on these 2D requests (up to 131 time
    # layers) it cuts the Krylov iterations by 1.1x to 3.8x
    srv = Server(slots=slots, prec=MIXED_FP32, tol_lin=1e-8, tol_nonlin=1e-8, lin_forcing=0.1, precond=1)
    recs = srv.run(reqs)
    out = summarize(recs)
    window = max(t for t, _ in reqs) - min(t for t, _ in reqs)
    out.update({"slots": slots, "arrival_rate_per_s": 20.0, "stream": f"first {n_requests} of 512 (seed 0)",
                "hbm_budget_bytes": srv.budget, "arrival_window_s": window,
                "sustained_req_per_s": out["completed"] / out["makespan_s"] if out["makespan_s"] > 0 else None,
                "unknowns_per_s": sum(p.unknowns for _, p in reqs) / out["makespan_s"] if out["makespan_s"] > 0
                else None})
    return out


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_region(torch, S, u1, u2, w, steps, warmup, tol):
    """Warm up, time exactly `steps` steps between synchronizations with the
    kernel profiler off, then run the same steps again with the profiler on
    for the per-kernel figures (HIP events around every launch)."""
    for _ in range(warmup):
        S.newton_step(u1, u2, w, True, tol)
        log("warmup step done")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    its = []
    rr = []
    for _ in range(steps):
        it, r, dinf = S.newton_step(u1, u2, w, True, tol)
        its.append(it)
        rr.append(r)
        log(f"step: {it} Krylov iterations, relres {r:.2e}")
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps
    S.profile(True)
    S.profile_read(reset=True)
    for _ in range(steps):
        S.newton_step(u1, u2, w, True, tol)
    torch.cuda.synchronize()
    prof = S.profile_read(reset=True)
    S.profile(False)
    log("profiled steps done")
    return ms, wall / steps * 1e3, its, rr, prof


def roofline(prof, steps, cfg=2):
    """Roofline entry of the kernel function with the largest summed duration:
    achieved rate from the algorithmic bytes (and flops, where recorded) of
    its launches over their HIP-event durations; the bound is the resource it
    uses the larger fraction of.  `traffic`: HBM bytes per launch measured
    with rocprofv3 counters (profiles/traffic.json), null when the kernel
    sources changed since."""
    fns = {k: v for k, v in prof.items() if k.startswith("fn:") and v[1] > 0}
    dom_name, (dom_ms, dom_n, dom_by, dom_fl) = max(fns.items(), key=lambda kv: kv[1][0])
    name = dom_name[3:]
    sec = dom_ms / 1e3
    f64 = "<f64>" in name
    hbm_frac = dom_by / sec / PEAK_HBM
    comp_frac, comp_peak, comp_bound = 0.0, None, None
    nonpacked_frac = None
    if dom_fl > 0:
        mfma = name.startswith("dense_mode_mfma") or name.startswith("time_core")
        # published peaks: FP64 vector and matrix 78.6, FP32 157.3 TFLOP/s
        comp_peak = PEAK_FP64 if f64 else PEAK_FP32
        comp_bound = "mfma" if mfma else "alu"
        comp_frac = dom_fl / sec / comp_peak
        if not f64 and not mfma:
            # FP32 vector code built without packed FP32 retires one FMA per
            # lane per cycle: 78.6 TFLOP/s is the rate it can reach
            nonpacked_frac = dom_fl / sec / PEAK_FP32_VALU
    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        from paper_2311_17500_amd.profiling import kernel_source_hash
        kern = t.get("configs", {}).get(str(cfg), {}).get("kernels", {})
        if t.get("kernel_source_sha256") == kernel_source_hash() and name in kern:
            traffic = kern[name]["hbm_bytes_per_launch"]
    except (OSError, ValueError):
        pass
    # the bound is the resource the kernel can saturate first: for FP32
    # vector code that is the non-packed rate
    comp_limit_frac = nonpacked_frac if nonpacked_frac is not None else comp_frac
    if comp_bound is not None and comp_limit_frac >= hbm_frac:
        roof = {"kernel": name, "bound": comp_bound, "achieved": dom_fl / sec / 1e12, "peak": comp_peak / 1e12,
                "unit": "TFLOP/s", "frac": comp_frac}
    else:
        roof = {"kernel": name, "bound": "hbm", "achieved": dom_by / sec / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": hbm_frac}
    roof.update({"traffic": traffic, "hbm_frac": hbm_frac, "compute_frac": comp_frac if comp_bound else None,
                 "compute_frac_vs_nonpacked_fp32": nonpacked_frac,
                 "nonpacked_fp32_peak_TFLOP_s": PEAK_FP32_VALU / 1e12 if nonpacked_frac is not None else None,
                 "avg_launch_ms": dom_ms / dom_n, "launches": dom_n, "alg_bytes_per_launch": dom_by / dom_n,
                 "alg_flops_per_launch": dom_fl / dom_n,
                 "kernels": {k[3:]: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps,
                                     "GB_per_s": (v[2] / (v[0] / 1e3) / 1e9) if v[0] > 0 else None,
                                     "TFLOP_per_s": (v[3] / (v[0] / 1e3) / 1e12) if v[0] > 0 and v[3] > 0 else None}
                             for k, v in sorted(fns.items(), key=lambda kv: -kv[1][0])},
                 "purpose_ms_per_step": {k: v[0] / steps for k, v in prof.items() if not k.startswith("fn:")}})
    return roof


def kernel_probe(cfg, reps):
    """For hardware-counter runs: a 1 GiB device copy (the calibration of the
    byte counters) followed by `reps` applications of the low-precision
    operator and preconditioner of the workload at the benchmark state."""
    import numpy as np
    import torch
    import st_workloads as W
    from paper_2311_17500_amd.binding import Solver, FP64, MIXED_FP32
    prob = W.config(cfg)
    mr = 16 if cfg == 4 else 48
    S = Solver(prob, prec=MIXED_FP32, tol_lin=1e-8, max_rank=mr)
    c0, _ = S.lift()
    u0 = torch.tensor(np.tile(c0, prob.n_t), dtype=torch.float64, device="cuda:0")
    u1, w = S.vec(S.full), S.vec(S.full)
    S.newton_step(u0, u1, w, True, 1e-8)
    S.linearize(u1, w, True)
    x = S.vec()
    x.copy_(torch.from_numpy(W.random_vector(prob.unknowns, 1)))
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    log("state ready; copy of 1 GiB")
    dst.copy_(src)
    torch.cuda.synchronize()
    for i in range(reps):
        S.apply_lowp(x)
        S.precond_lowp(x)
        torch.cuda.synchronize()
        log(f"probe rep {i} done")
    print(json.dumps({"kernel_probe": True, "config": cfg, "reps": reps, "copy_bytes": 2 * (1 << 30)}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg):
    """The oracle as it stands on the host cores: one Newton step (explicit
    assembly + sparse LU) of the same physics on a reduced mesh."""
    import numpy as np
    import st_workloads as W
    from oracle import solver as osolver
    from oracle.spacetime import SpaceTime
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    base = W.config(cfg)
    nel = {0: 32, 1: 10, 2: 6, 4: 5}[cfg]
    prob = W.tiny(base.d, base.p_s, nel, nel_t=nel, sigma=base.sigma, u0_radius=base.u0_radius,
                  u0_center=base.u0_center, u0_kind=base.u0_kind)
    st = SpaceTime(prob)
    u0 = np.tile(st.lift(), st.n[-1])
    t0 = time.perf_counter()
    w = st.w_update_explicit(u0)
    lin = osolver.linearize(st, u0, w)
    J = st.assemble_J(lin.coef_q, lin.theta_q)
    r = st.residual(u0, w, lin.theta_q)
    import scipy.sparse.linalg as spla
    spla.splu(J.tocsc()).solve(-r)
    dt = time.perf_counter() - t0
    return {"value": prob.dof / dt, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "sample": (f"one oracle Newton step (explicit sparse assembly by Gauss quadrature + scipy splu) of "
                       f"the same physics at d={prob.d}, p={prob.p_s}, {nel}^{prob.d}x{nel} elements "
                       f"({prob.dof} DOF) in {dt:.2f} s; splu is single-threaded, BLAS pool {cores}")}


def bench_config(torch, W, cfg, precs, steps, warmup, tol, max_rank, solve_only_too, precond=0):
    """Time one workload in the given precisions at the fixed state u^1 (one
    FP64 Newton step from the lifted datum).  One large context at a time."""
    import numpy as np
    from paper_2311_17500_amd.binding import Solver, FP64, MIXED_FP32, MIXED_BF16
    prob = W.config(cfg)
    codes = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}
    S64 = Solver(prob, prec=FP64, tol_lin=tol, max_rank=max_rank, precond=precond)
    c0, _ = S64.lift()
    u0 = torch.tensor(np.tile(c0, prob.n_t), dtype=torch.float64, device="cuda:0")
    u1, w = S64.vec(S64.full), S64.vec(S64.full)
    log(f"config {cfg}: {prob.dof} DOF, workspace {S64.workspace_bytes / 1e9:.1f} GB (FP64)")
    S64.newton_step(u0, u1, w, True, tol)
    del u0
    log("state u1 ready")
    u2 = S64.vec(S64.full)
    torch.cuda.synchronize()

    def solve_only(S):
        """The linear solve alone (the Krylov part of the step) on the same system."""
        S.linearize(u1, w, True)
        b = -S.residual(u1, w)
        x = S.vec()
        for _ in range(warmup):
            S.krylov(b, tol, x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            _, its, rr = S.krylov(b, tol, x)
        e1.record()
        torch.cuda.synchronize()
        sm = e0.elapsed_time(e1) / steps
        return {"ms": sm, "dof_per_s": prob.dof / (sm / 1e3), "krylov_iters": its, "relres": rr}

    out = {}
    for prec in precs:
        if prec == "fp64":
            S = S64
        else:
            if S64 is not None and S64.ctx:
                S64.close()
                S64.ws = None
                torch.cuda.empty_cache()
            S = Solver(prob, prec=codes[prec], tol_lin=tol, max_rank=max_rank, precond=precond)
        ms, wall, its, rr, prof = time_region(torch, S, u1, u2, w, steps, warmup, tol)
        r = dict(ms=ms, wall=wall, its=its, rr=rr, prof=prof)
        log(f"config {cfg} {prec} Newton steps timed: {ms:.1f} ms")
        if solve_only_too:
            r["solve"] = solve_only(S)
            log(f"config {cfg} {prec} solve-only timed")
        out[prec] = r
        if S is not S64:
            S.close()
            S.ws = None
            torch.cuda.empty_cache()
    if S64.ctx:
        S64.close()
        S64.ws = None
    torch.cuda.empty_cache()
    return prob, out


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Context for the HBM fractions: read + write bytes per second of a
    plain device-to-device copy of 1 GiB on this GPU (torch's copy kernel)."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def summary(prob, cfg, prec, r, steps):
    """Compact record of one measured configuration (extra keys of the line)."""
    roof = roofline(r["prof"], steps, cfg)
    top = dict(list(roof["kernels"].items())[:6])
    return {"workload": f"config{cfg}: d={prob.d} p={prob.p_s} {'x'.join(map(str, prob.nel_s))}x{prob.nel_t} "
                        f"elements, {prob.dof} DOF, {prec}",
            "dof_per_s": prob.dof / (r["ms"] / 1e3), "ms_per_step": r["ms"], "krylov_iters_per_step": r["its"][0],
            "final_relres": r["rr"][-1],
            "dominant_kernel": {k: roof[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac",
                                                     "hbm_frac", "compute_frac", "compute_frac_vs_nonpacked_fp32",
                                                     "avg_launch_ms", "traffic")},
            "top_kernels": top}


def compare_su(torch, W):
    """Galerkin vs SU with the paper's fixed-point scheme (Section 3.1 with
    the stopping rule of Section 4) on config 1 and on a source-driven
    variant of it (zero datum, a disc stimulus during [0.1, 0.2], time knots
    clustered at the source's on/off times), on the paper's 2D setting, and
    SUPG with and without shock capturing (c = 0.1, h in physical time) on
    C^0 time splines in that setting:
    fixed-point iterations, Krylov iterations per fixed-point iteration,
    extremes of u, wall time."""
    from paper_2311_17500_amd.binding import Solver, FP64, StIgaError
    base = W.config(1)
    src = dict(base.__dict__)
    src.update(u0_kind=0, f_kind=1, f_center=(0.0, 0.0, 0.0), f_radius=0.1, f_t0=0.1, f_t1=0.2, f_amp=5.0)
    # the paper's 2D test (Section 4.2) with its Rogers-McCulloch set, C_m = 1,
    # D = 1e-4, T = 300, p = 3 and its meshes (2^-6 x 2^-3 x 2^-5) and moving
    # Gaussian source during [90, 100], on the rectangle [0, 1.5] x [0, 0.125]
    # (affine map) standing in for the elliptic ring, whose parametrization
    # the paper does not give
    L1, L2, Tp = 1.5, 0.125, 300.0
    paper = W.Problem(d=2, p_s=3, p_t=3, nel_s=(64, 8), nel_t=32, sigma=(1e-4, 1e-4), T=Tp, Cm=1.0,
                      a=0.13, b=0.013, c1=0.26, c2=0.1, de=1.0, u0_kind=0,
                      f_kind=2, f_center=(0.0, L2 / 2, 0.0), f_velocity=(8.0 / 15.0 * L1 / Tp, 0.0, 0.0),
                      f_kappa=500.0, f_amp=0.25, f_t0=90.0, f_t1=100.0,
                      map_kind=(1, 1, 0), map_param=((0.0, L1, 0.0), (0.0, L2, 0.0), (0.0, 1.0, 0.0)))
    # the paper's C^0 comparison (Section 4.2.2): the same 2D setting with C^0
    # cubic splines in time on 12 elements (N_t = 36), SUPG + shock capturing
    paper_c0 = W.Problem(**{**paper.__dict__, "nel_t": 12})
    std = (("su", 1, 0.0), ("galerkin", 0, 0.0))
    cases = [("config1", base, None, std),
             ("config1_source_clustered_time", W.Problem(**src),
              W.clustered_time_knots(base.nel_t, base.p_t, [0.1, 0.2], 0.004), std),
             ("paper2d_uniform_time", paper, None, std),
             ("paper2d_clustered_time", paper, W.clustered_time_knots(32, 3, [90.0 / Tp, 100.0 / Tp], 0.003), std),
             ("paper2d_c0_time", paper_c0, W.c0_time_knots(12, 3),
              (("supg_sc", 2, 0.1), ("supg", 2, 0.0), ("galerkin", 0, 0.0)))]
    out = {}
    for name, prob, tk, modes in cases:
        knots = None
        if tk is not None:
            knots = prob.uniform_knots()
            knots[prob.d] = tk
        for mode, su, sc_c in modes:
            S = Solver(prob, knots=knots, prec=FP64, su=su, outer=2, alpha=0.5, tol_nonlin=1e-4, tol_lin=1e-8,
                       max_outer=300, sc_c=sc_c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status = "ok"
            try:
                u, w, rep = S.solve()
            except StIgaError as e:
                status = str(e)
                rep = None
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec = {"status": status, "seconds": dt}
            if rep is not None:
                n = rep.outer_iters
                rec.update({"fixed_point_iters": n, "krylov_total": rep.krylov_total,
                            "krylov_per_fixed_point": rep.krylov_total / max(n, 1),
                            "theta_rank_last": rep.rank_theta[min(n, 64) - 1] if su == 1 else 0,
                            "u_max": float(u.abs().max()), "u_min": float(u.min())})
            out[f"{name}_{mode}"] = rec
            log(f"{name} su={su}: {rec}")
            S.close()
            torch.cuda.empty_cache()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported "
              f"(the multi-GPU layout is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import st_workloads as W
    if a.kernel_probe > 0:
        kernel_probe(a.config, a.kernel_probe)
        return
    if a.compare_su:
        print(json.dumps({"compare_su": compare_su(torch, W)}), flush=True)
        return
    if a.serve:
        s = serving(512, a.serve_slots)
        print(json.dumps({"metric": "p50/p99 solve latency, 512-request serving stream (config 3)",
                          "value": s["p99_latency_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
                          "data": "synthetic", "config": {"workload": "config3: 512 seeded 2D solves at 20 req/s"},
                          "serving": s}), flush=True)
        return

    if a.max_rank is None:
        a.max_rank = 16 if a.config == 4 else 48
    precs = [a.prec] if (a.prec == "fp64" or a.no_fp64_compare) else ["fp64", a.prec]
    prob, res = bench_config(torch, W, a.config, precs, a.steps, a.warmup, a.tol, a.max_rank, True, a.precond)
    main_r = res[a.prec]
    ms = main_r["ms"]
    value = prob.dof / (ms / 1e3)
    roof = roofline(main_r["prof"], a.steps, a.config)
    roof["device_copy_GB_per_s"] = copy_bandwidth(torch)
    out = {
        "metric": "space-time DOF/s to rel. residual 1e-8 (mixed vs FP64); p50/p99 solve latency",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed_fp32": "f32+f64", "mixed_bf16": "bf16+f64"}[a.prec],
        "data": "synthetic",
        "config": {"workload": f"config{a.config}: d={prob.d} p={prob.p_s} "
                               f"{'x'.join(map(str, prob.nel_s))}x{prob.nel_t} elements, "
                               f"{prob.dof} DOF ({prob.unknowns} unknowns), {a.prec}",
                   "dof": prob.dof, "unknowns": prob.unknowns, "precision": a.prec,
                   "tol": a.tol, "precond": ["fast diagonalization", "banded time"][a.precond],
                   "step": "one Newton iteration (linearize + residual + FGMRES/FD to 1e-8)"},
        "krylov_iters_per_step": main_r["its"][0], "final_relres": main_r["rr"][-1],
        "wall_ms_per_step": main_r["wall"],
        "roofline": roof,
    }
    solve = {p: r["solve"] for p, r in res.items()}
    if len(solve) == 2:
        solve["speedup_mixed_vs_fp64"] = solve["fp64"]["ms"] / solve[a.prec]["ms"]
    out["linear_solve_only"] = solve
    if "fp64" in res and a.prec != "fp64":
        f = res["fp64"]
        out["fp64_dof_per_s"] = prob.dof / (f["ms"] / 1e3)
        out["fp64_ms_per_step"] = f["ms"]
        out["fp64_krylov_iters_per_step"] = f["its"][0]
        out["speedup_vs_fp64"] = f["ms"] / ms
    if not a.no_extras and a.config == 2:
        # the other precision of the same workload and the largest one-GPU workload
        extras = {}
        p2, r2 = bench_config(torch, W, 2, ["mixed_bf16"], a.steps, a.warmup, a.tol, 48, False)
        extras["config2_mixed_bf16"] = summary(p2, 2, "mixed_bf16", r2["mixed_bf16"], a.steps)
        p4, r4 = bench_config(torch, W, 4, ["mixed_fp32"], 2, 1, a.tol, 16, False)
        extras["config4_mixed_fp32"] = summary(p4, 4, "mixed_fp32", r4["mixed_fp32"], 2)
        out["extra_workloads"] = extras
    if a.serve_requests > 0:
        log("serving sample")
        out["serving"] = serving(a.serve_requests, a.serve_slots)
    if not a.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(a.config)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
