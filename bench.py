"""Benchmark: 512^3 FP64 Jacobi, T = 100 sweeps, temporally blocked vs plain.

Default workload (one JSON line): one step = T = 100 sweeps of the 512^3
interior (514^3 arrays) FP64 grid through jacobi_tblock at the library's
default blocking (--autotune: the autotuner's pick); inputs are resident in HBM before the timed region and
consecutive steps continue the iteration (level 100 of one step is level 0
of the next; the work does not depend on the values).

  value         GLUP/s of the blocked run (512^3 * 100 / time per step)
  roofline      the blocked kernel against HBM: algorithmic bytes per launch
                (16 B per cell per pass, one read and one write of each cell)
                over its average launch duration (HIP events on the stream the
                kernels run on), against the 8 TB/s HBM peak; `traffic` is the
                measured HBM traffic per launch from the committed rocprofv3
                summary of that kernel (or --traffic), null once the kernel
                sources differ from those it was measured on
  plain         the plain one-pass-per-sweep kernel under the same protocol
  cpu_baseline  the CPU oracle on a bounded sample of the same workload

Other workloads (--workload): `batched` (64 grids, edges log-uniform in
[32, 256], T = 50, one persistent launch), `adjoint` (256^3, T = 32,
autograd forward + backward and the adjoint call alone), `refine` (768^3
Laplace solve, FP32 inner / FP64 outer, vs all-FP64 Jacobi; runs many
minutes, or --refine-outer K for a bounded run), `pipelined` (512^3, T = 100,
by the pipelined schedule, with the looseness sweep of Eq. 3), `compressed`
(512^3, T = 100, in one array), `lbm` (D3Q19 lattice Boltzmann, 256^3, FP64
and FP32), `fp32` (the blocked pass in FP32 at 512^3, T = 100, and with a
right-hand side at 768^3, T = 50, every depth).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X: 256 CUs at up to 2.4 GHz; one 64-lane VALU instruction per CU and
# clock (FP64 FMA included: 78.6 TFLOP/s); LDS 128 B per CU and clock
CUS, CLOCK_HZ = 256, 2.4e9
LDS_PEAK_TBS = CUS * CLOCK_HZ * 128 / 1e12
# bytes per lane and LDS instruction of the blocked pass's stream step (its
# loop issues 16 ds_read_b64, 8 ds_read2st64_b64 and 4 ds_write2st64_b64:
# 320 B per lane over 28 instructions)
LDS_BYTES_PER_LANE_INST = 320 / 28
PROFILES = os.path.join(ROOT, "profiles")


def profile_figures(name, kernel_fragment):
    """Figures of a committed rocprofv3 summary (profiles/NAME.md) when it was
    measured on this kernel instance with the current kernel sources, else
    None (the kernel changed since the counters were taken)."""
    from paper_0912_4506_amd import profiling
    fig = profiling.read_figures(os.path.join(PROFILES, name))
    if not fig or kernel_fragment not in str(fig.get("kernel", "")):
        return None
    if fig.get("kernel_source_sha") != profiling.kernel_source_hash():
        return None
    return fig
METRIC = "GLUP/s & % roofline, 512³ FP64 Jacobi T=100: temporal-blocked vs plain"
# why a depth the workload names has no kernel
DEPTH_REFUSAL = {16: " (the blocked pass keeps about two values per cell and level in "
                     "registers, 4t VGPRs per cell in FP64: depth 16 would need 64 per cell, and "
                     "depth 8 already spills on blocks with useful halo overhead)"}


def dominant_depth(T, passes):
    """The depth most of the passes of a T-sweep run run at (the library
    splits T into passes whose depths differ by at most one)."""
    base, rem = divmod(T, passes)
    return base + 1 if rem > passes - rem else base


def ensure_built():
    from paper_0912_4506_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def time_steps(fn, steps, warmup):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per step


def copy_bandwidth(jac, nbytes=2 << 30, reps=5):
    """M_s (Eq. 2): the library's copy kernel over two nbytes arrays (beyond
    the 256 MB last-level cache); bytes read + written per second."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ms = time_steps(lambda: jac.copy(dst, src), reps, 2)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(u, T, lups_per_sweep, target_s=12.0):
    """The CPU oracle, as it stands, on the host cores: the whole grid for as
    many of the T sweeps as fit about target_s seconds."""
    import oracle
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.sweeps(u, 2)
    t1 = time.perf_counter()
    oracle.sweeps(u, 1)
    t2 = time.perf_counter()
    per_sweep = max((t1 - t0) - (t2 - t1), 1e-3)
    sweeps = max(1, min(T, int(target_s / per_sweep)))
    t0 = time.perf_counter()
    oracle.sweeps(u, sweeps)
    dt = time.perf_counter() - t0
    # the same oracle on one thread: one sweep's time, as the difference of a
    # two-sweep and a one-sweep run (allocation and first touch cancel)
    t1 = time.perf_counter()
    oracle.sweeps(u, 2, nthreads=1)
    t2 = time.perf_counter()
    oracle.sweeps(u, 1, nthreads=1)
    dt1 = max((t2 - t1) - (time.perf_counter() - t2), 1e-6)
    oracle.max_threads(cores)     # the oracle's thread count is process-wide: restore it
    # the paper's baseline model on the host (Eq. 2): P0 = M_s / 16 B with the
    # host's own copy bandwidth
    ms_host = oracle.copy_bandwidth(1 << 27, 5)
    n = round(u.shape[0] - 2)
    value = lups_per_sweep * sweeps / dt / 1e9
    return {"value": round(value, 4), "unit": "GLUP/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{n}^3 FP64 grid, {sweeps} of the {T} sweeps, one run ({dt:.1f} s)",
            "single_thread": round(lups_per_sweep / dt1 / 1e9, 4),
            "host_copy_gbs": round(ms_host / 1e9, 1),
            "p0_host_glups": round(ms_host / 16 / 1e9, 3),
            "frac_of_p0_host": round(value / (ms_host / 16 / 1e9), 3)}


def bench_metric(args):
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    N, T = 512, 100
    u = inputs.grid(N, N, N, seed=0)
    a = torch.from_numpy(u).to("cuda")
    b = torch.empty_like(a)
    lups = N ** 3 * T
    cell_bytes = 16 * N ** 3  # one read + one write of each cell per pass

    if args.autotune:
        # the library's autotuner picks the blocking (every shape and depth)
        (t, bx, by, w), _ = jac.autotune(a, b, T, tmax=args.tmax, reps=1)
        a.copy_(torch.from_numpy(u))
    else:
        # the library's default blocking for this grid (or a pinned choice)
        t = args.t or jac.default_tile(a.shape, T)[0]
        d = jac.default_tile(a.shape, T, t)
        bx, by, w = (args.bx, args.by, args.waves) if args.bx else (d[1], d[2], d[4])
    state = {"a": a, "b": b}

    def step(t=t, bx=bx, by=by, w=w):
        out = jac.tblock(state["a"], state["b"], T, t=t, bx=bx, by=by, waves=w)
        if out is state["b"]:
            state["a"], state["b"] = state["b"], state["a"]

    ms = time_steps(step, args.steps, args.warmup)
    passes = math.ceil(T / t)
    kernel_ms = ms / passes
    tile = jac.default_tile(a.shape, T, t)

    by_depth = {}
    if args.depths:
        from paper_0912_4506_amd._lib import JacobiError
        for d in [int(x) for x in args.depths.split(",") if x]:
            best, refusal = None, None
            for (sx, sy, sw) in jac.tile_menu(torch.float64):
                try:
                    dms = time_steps(lambda: jac.tblock(state["a"], state["b"], T, t=d, bx=sx, by=sy,
                                                        waves=sw), 1, 1)
                except JacobiError as e:
                    refusal = str(e)
                    continue
                if best is None or dms < best[0]:
                    best = (dms, sx, sy, sw)
            if best:
                by_depth[str(d)] = {"glups": round(lups / (best[0] * 1e-3) / 1e9, 1),
                                    "tile": [best[1], best[2]], "waves": best[3]}
            else:
                by_depth[str(d)] = ("refused: " + (refusal or "no block shape runs at this depth")
                                    + DEPTH_REFUSAL.get(d, ""))

    plain = None
    if not args.no_plain:
        def pstep():
            out = jac.plain(state["a"], state["b"], T)
            if out is state["b"]:
                state["a"], state["b"] = state["b"], state["a"]
        pms = time_steps(pstep, max(1, args.steps // 2), 1)
        plain = {"glups": round(lups / (pms * 1e-3) / 1e9, 2), "ms_per_step": round(pms, 3),
                 "kernel_ms": round(pms / T, 4),
                 "achieved_gbs": round(cell_bytes / (pms / T * 1e-3) / 1e9, 1)}

    del a, b, state
    torch.cuda.empty_cache()
    ms_copy = copy_bandwidth(jac)
    achieved = cell_bytes / (kernel_ms * 1e-3) / 1e9
    glups = lups / (ms * 1e-3) / 1e9
    # the kernel instance this blocking runs, and its committed profile
    # (rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by the copy kernel's, and the SQ
    # instruction counters), used only while the kernel sources are unchanged
    inst = f"tblock_kernel<double, {t}, {bx // 64}, {by // w}, {w}, 0>"
    prof_name = f"tblock_f64_t{t}_{bx}x{by}_512cubed.md"
    fig = profile_figures(prof_name, inst)
    traffic = fig.get("traffic_gb_per_launch") if fig else None
    if args.traffic:
        traffic = float(args.traffic)
    from paper_0912_4506_amd import perf_model
    t_eff = perf_model.t_eff(T, t)
    p_t = perf_model.roofline(ms_copy * 1e9, T, t) / 1e9          # M_s t_eff / 16 B (Eq. 2)
    lups_launch = N ** 3 * t_eff
    secondary = {"p_t": {"t_eff": t_eff, "ms_gbs": round(ms_copy, 1), "glups": round(p_t, 1),
                         "frac": round(glups / p_t, 4)}}
    # Eq. 5 as a prediction: speedup over P0 of t_eff updates per transfer when
    # the levels share an on-chip path of rate M_c' (the LDS bandwidth here;
    # on a GPU the chip saturates HBM, so M_s,1 = M_s)
    sp = perf_model.speedup(ms_copy, ms_copy, LDS_PEAK_TBS * 1e3, t_eff)
    secondary["eq5"] = {"mc_prime_tbs": round(LDS_PEAK_TBS, 1), "speedup_over_p0": round(sp, 3),
                        "predicted_glups": round(sp * ms_copy / 16, 1),
                        "measured_over_predicted": round(glups / (sp * ms_copy / 16), 3)}
    if fig and "sq_insts_valu_per_launch" in fig:
        valu = fig["sq_insts_valu_per_launch"]
        per_lup = valu * 64 / lups_launch                           # lane instructions per update
        ceiling = CUS * CLOCK_HZ * 64 / per_lup / 1e9
        secondary["valu"] = {"wave_insts_per_launch": int(valu), "lane_insts_per_lup": round(per_lup, 2),
                             "ceiling_glups": round(ceiling, 1), "frac": round(glups / ceiling, 4),
                             "peak": "256 CUs x 64 lanes x 2.4 GHz"}
    if fig and "sq_insts_lds_per_launch" in fig:
        lds_bytes = fig["sq_insts_lds_per_launch"] * 64 * LDS_BYTES_PER_LANE_INST
        lds_tbs = lds_bytes / (kernel_ms * 1e-3) / 1e12
        secondary["lds"] = {"bytes_per_launch": int(lds_bytes), "achieved_tbs": round(lds_tbs, 2),
                            "peak_tbs": round(LDS_PEAK_TBS, 1), "frac": round(lds_tbs / LDS_PEAK_TBS, 4)}
    line = {
        "metric": METRIC,
        "value": round(glups, 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: uniform [0,1) interior and shell, numpy default_rng(0)",
        "config": {"workload": "jacobi3d 512^3 interior (514^3 arrays), FP64, T=100, Dirichlet shell",
                   "t": t, "tile_bx_by": [bx, by], "waves": w, "kchunk": tile[3],
                   "passes": passes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "GB per launch",
                     "algorithmic_bytes_per_launch": cell_bytes,
                     "kernel": inst, "profile": ("profiles/" + prof_name) if fig else None,
                     "profile_median_us": fig.get("median_us") if fig else None,
                     "bench_us_per_launch": round(kernel_ms * 1e3, 1),
                     **secondary},
        "plain": plain,
        "by_depth": by_depth,
        "copy_bandwidth_gbs": round(ms_copy, 1),
        "p0_glups": round(ms_copy / 16, 1),
        "vs_plain": round((lups / (ms * 1e-3) / 1e9) / plain["glups"], 3) if plain else None,
        "vs_p0": round((lups / (ms * 1e-3) / 1e9) / (ms_copy / 16), 3),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(u, T, N ** 3)
    return line


def bench_batched(args):
    import numpy as np
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    edges = inputs.batch_edges(64, seed=0, cubic=not args.noncubic)
    us = [inputs.batch_grid(e, m, seed=0) for m, e in enumerate(edges)]
    a = [torch.from_numpy(x).to("cuda") for x in us]
    b = [torch.empty_like(x) for x in a]
    T = 50
    lups = sum(nx * ny * nz for nx, ny, nz in edges) * T
    if args.t and args.bx:
        t, bx, by, w = args.t, args.bx, args.by, args.waves
    else:
        (t, bx, by, w), _ = jac.autotune_batch(a, b, [T] * 64, reps=1)
    plan = jac.BatchPlan(a, b, [T] * 64, t=t, bx=bx, by=by, waves=w)
    # cells the blocks compute per valid cell: every pass of a grid streams
    # nti*bx x ntj*by columns through the planes of each k chunk [k0, k1)
    # plus depth planes on either side (k from max(k0 - t, 0) to k1 + t - 1)
    computed = valid = 0
    per_grid = []
    for G in plan.geometry():
        steps = 0
        for q in range(G["nkc"]):
            k0 = 1 + q * G["kchunk"]
            k1 = min(k0 + G["kchunk"], G["nz"] + 1)
            steps += (k1 + G["t"]) - max(k0 - G["t"], 0)
        c = G["nti"] * bx * G["ntj"] * by * steps
        v = G["nx"] * G["ny"] * G["nz"]
        computed += c * G["passes"]
        valid += v * G["passes"]
        per_grid.append(round(c / v, 2))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run("relaxed")
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run("relaxed")
    ms = time_steps(g.replay, args.steps, args.warmup)
    lms = pms = tms = None
    if not args.relaxed_only:
        lms = time_steps(lambda: plan.run("lockstep"), args.steps, 1)

        def seq_plain():      # per-grid plain calls, one after another
            for x, y in zip(a, b):
                jac.plain(x, y, T)
        pms = time_steps(seq_plain, max(1, args.steps // 2), 1)

        def seq_tb():
            for x, y in zip(a, b):
                jac.tblock(x, y, T, t=t, bx=bx, by=by, waves=w)
        tms = time_steps(seq_tb, max(1, args.steps // 2), 1)
    del a, b, plan, g
    torch.cuda.empty_cache()
    ms_copy = copy_bandwidth(jac)
    passes = math.ceil(T / t)
    achieved = 16 * (lups / T) * passes / (ms * 1e-3) / 1e9     # 16 B per cell and pass
    return {"metric": "batched GLUP/s, 64 grids (edges log-uniform in [32,256]) FP64 T=50",
            "value": round(lups / (ms * 1e-3) / 1e9, 2), "unit": "GLUP/s", "n_gpus": 1,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "copy_bandwidth_gbs": round(ms_copy, 1),
                         "p_t_glups": round(ms_copy * (T / passes) / 16, 1)},
            "computed_per_valid_cell": round(computed / valid, 3),
            "computed_per_valid_cell_by_grid": per_grid,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "64 cubic grids" if not args.noncubic else "64 non-cubic grids",
                       "interior_cells": int(lups // T), "t": t, "tile_bx_by": [bx, by], "waves": w,
                       "graph": True},
            "lockstep_glups": round(lups / (lms * 1e-3) / 1e9, 2) if lms else None,
            "sequential_plain_glups": round(lups / (pms * 1e-3) / 1e9, 2) if pms else None,
            "sequential_tblock_glups": round(lups / (tms * 1e-3) / 1e9, 2) if tms else None}


def bench_adjoint(args):
    """autograd forward + backward at 256^3, T = 32 (the backward is the
    library's adjoint pass), FP64 and FP32, with and without checkpoints every
    8 levels; and the adjoint call alone, whose blocked trace-mode pass is the
    dominant kernel: its roofline at 16 B per cell and pass (FP64)."""
    import math
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac
    from paper_0912_4506_amd.autograd import JacobiT, checkpoints

    n, T, every = 256, 32, 8
    out = {"metric": "autograd forward+backward, 256^3, T=32, checkpoints every 8 levels",
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": False, "dtype": "f64",
           "data": "synthetic: uniform [0,1) grid, loss sum(w * A_T^2) with uniform [0,1) w",
           "config": {"workload": f"jacobi3d {n}^3, T={T}, autograd with checkpoints every {every}"},
           "results": {}}
    for dt in (torch.float64, torch.float32):
        name = "f64" if dt == torch.float64 else "f32"
        u = torch.from_numpy(inputs.grid(n, n, n, seed=0)).to("cuda", dt)
        w = torch.from_numpy(inputs.adjoint_weights(n, n, n, seed=0)).to("cuda", dt)

        def fwd_bwd_ckpt():
            x = u.detach().requires_grad_(True)
            A = checkpoints(x, T, every)[-1]
            (w * A * A).sum().backward()

        def fwd_bwd():
            x = u.detach().requires_grad_(True)
            A = JacobiT.apply(x, T)
            (w * A * A).sum().backward()

        cms = time_steps(fwd_bwd_ckpt, args.steps, args.warmup)
        ms = time_steps(fwd_bwd, args.steps, args.warmup)
        a = u.clone()
        b = torch.empty_like(a)
        pms = time_steps(lambda: jac.plain(a, b, T), args.steps, 1)
        # the adjoint call alone at the library's default blocking
        lam = w.clone()
        lb = torch.empty_like(lam)
        ws = jac.adjoint_workspace(lam)
        ams = time_steps(lambda: jac.adjoint(lam, lb, T, ws=ws), args.steps, args.warmup)
        t = jac.default_tile(lam.shape, T, 0, dtype=dt, adjoint=True)[0]
        passes = math.ceil(T / t)
        pass_bytes = 2 * n ** 3 * lam.element_size()
        achieved = pass_bytes / (ams / passes * 1e-3) / 1e9
        out["results"][name] = {
            "fwd_bwd_checkpointed_ms": round(cms, 3), "fwd_bwd_ms": round(ms, 3),
            "plain_forward_ms": round(pms, 3),
            "ratio_to_plain_forward": round(cms / pms, 3),
            "adjoint_ms": round(ams, 3), "adjoint_t": t, "adjoint_passes": passes,
            "adjoint_glups": round(n ** 3 * T / (ams * 1e-3) / 1e9, 1),
            "adjoint_achieved_gbs": round(achieved, 1)}
        del u, w, a, b, lam, lb, ws
        torch.cuda.empty_cache()
    f64 = out["results"]["f64"]
    out["value"] = f64["fwd_bwd_checkpointed_ms"]
    out["ms_per_step"] = f64["fwd_bwd_checkpointed_ms"]
    # HBM traffic of the FP64 trace-mode pass from its committed profile
    # (rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by the copy kernel's), for the
    # depth most passes run at
    out["copy_bandwidth_gbs"] = round(copy_bandwidth(jac), 1)
    t, bx, by, _, w = jac.default_tile((n + 2,) * 3, T, 0, dtype=torch.float64, adjoint=True)
    passes = math.ceil(T / t)
    fig = profile_figures(f"adjoint_f64_{n}cubed.md",
                          f"tblock_kernel<double, {dominant_depth(T, passes)}, {bx // 64}, "
                          f"{by // w}, {w}, 2>")
    out["roofline"] = {"bound": "hbm", "kernel": "the adjoint's blocked trace-mode pass (FP64)",
                       "achieved": f64["adjoint_achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(f64["adjoint_achieved_gbs"] / HBM_PEAK_GBS, 4),
                       "traffic": fig.get("traffic_gb_per_launch") if fig else None,
                       "traffic_unit": "GB per launch",
                       "algorithmic_bytes_per_launch": 2 * n ** 3 * 8}
    return out


def bench_pipelined(args):
    """512^3 FP64, T = 100 by pipelined temporal blocking (the team pipeline
    with relaxed synchronisation, one persistent launch).  Two parts:
      * the looseness sweep of the paper's relaxed-synchronisation study
        (Eq. 3): for a few (team, sweeps per item, k chunk) settings, the
        upper distance du in {1 (lock-step with dl = 1), 2, 4, none} and a
        team delay of 8 chunks;
      * the fastest of a small grid of (team, sweeps per item, k chunk) with
        no upper bound,
    against the overlapped-tile default and the plain kernel on the same grid."""
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    N, T = 512, 100
    u = inputs.grid(N, N, N, seed=0)
    a = torch.from_numpy(u).to("cuda")
    b = torch.empty_like(a)
    lups = N ** 3 * T

    def measure(team, t, kc, dl=1, du=0, dt=0):
        try:
            plan = jac.PipelinePlan(a, b, T, team=team, t=t, kchunk=kc, dl=dl, du=du, dt=dt)
        except Exception as e:          # a refused shape: skip it
            print(f"  team {team} t {t} kchunk {kc}: {e}", file=sys.stderr)
            return None
        ms = time_steps(lambda: plan.run("relaxed"), max(1, args.steps // 2), 1)
        if plan.wait_error():
            raise RuntimeError("a relaxed-mode wait gave up")
        row = {"team": team, "t": t, "kchunk": kc, "dl": dl, "du": du if du else "none", "dt": dt,
               "glups": round(lups / (ms * 1e-3) / 1e9, 1)}
        print(f"  {row}", file=sys.stderr, flush=True)
        return row

    looseness = []
    for team, t, kc in ((4, 1, 16), (8, 1, 32), (4, 2, 32), (4, 4, 64)):
        rows = [measure(team, t, kc, 1, du) for du in (1, 2, 4, 0)]
        rows.append(measure(team, t, kc, 1, 2, 8))
        rows = [r for r in rows if r]
        if rows:
            lock = rows[0]["glups"] if rows[0]["du"] == 1 else None
            looseness.append({"team": team, "t": t, "kchunk": kc,
                              "glups_by_du": {str(r["du"]): r["glups"] for r in rows if r["dt"] == 0},
                              "glups_du2_dt8": next((r["glups"] for r in rows if r["dt"] == 8), None),
                              "best_vs_lockstep": round(max(r["glups"] for r in rows) / lock, 3)
                              if lock else None})
    rows = []
    for team in (1, 2, 4, 8):
        for t in (1, 2, 4):
            for kc in (16, 32, 64, 128):
                r = measure(team, t, kc)
                if r:
                    rows.append(r)
    best = max(rows, key=lambda r: r["glups"])
    bms = time_steps(lambda: jac.tblock(a, b, T), args.steps, 1)
    pms = time_steps(lambda: jac.plain(a, b, T), max(1, args.steps // 2), 1)
    # one persistent launch runs every pass: algorithmic traffic 16 B per
    # cell and pass, over the launch's time
    passes = math.ceil(T / best["t"])
    achieved = 16 * N ** 3 * passes / (lups / (best["glups"] * 1e9)) / 1e9
    return {"metric": "GLUP/s, 512^3 FP64 Jacobi T=100, pipelined temporal blocking", "unit": "GLUP/s",
            "value": best["glups"], "higher_is_better": True, "n_gpus": 1, "dtype": "f64",
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(lups / (best["glups"] * 1e9) * 1e3, 3),
            "data": "synthetic: uniform [0,1) interior and shell, numpy default_rng(0)",
            "roofline": {"bound": "hbm", "kernel": "batched_kernel, pipelined order (one launch, all passes)",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                         "algorithmic_bytes_per_launch": 16 * N ** 3 * passes},
            "config": {"workload": "jacobi3d 512^3 interior, FP64, T=100", **best},
            "overlapped_tiles_glups": round(lups / (bms * 1e-3) / 1e9, 1),
            "plain_glups": round(lups / (pms * 1e-3) / 1e9, 1),
            "looseness": looseness, "candidates": rows}


def bench_compressed(args):
    """512^3 FP64, T = 100 in one array (the compressed grid) at depths 4, 5
    and 6 with the library's default block for each (--t pins one), against
    jacobi_tblock with the same blocking on two arrays.  Each step runs from
    frame 0 again (the work does not depend on the values)."""
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    N, T = 512, 100
    u = inputs.grid(N, N, N, seed=0)
    lups = N ** 3 * T
    rows = []
    for t in ([args.t] if args.t else [4, 5, 6]):
        d = jac.default_tile((N + 2,) * 3, T, t)
        bx, by, w = (args.bx, args.by, args.waves) if args.bx else (d[1], d[2], d[4])
        arr = torch.empty(jac.compressed_shape(N, N, N, t), dtype=torch.float64, device="cuda")
        jac.compressed_frame(arr, t, 0).copy_(torch.from_numpy(u))
        run = jac.Compressed(arr, T, t, bx=bx, by=by, waves=w)
        ms = time_steps(run.run, args.steps, args.warmup)
        torch.cuda.synchronize()
        if run.wait_error():
            raise RuntimeError("a compressed-grid wait gave up")
        comp_bytes = arr.numel() * 8 + run.ws_view.numel()
        del arr, run
        torch.cuda.empty_cache()
        a = torch.from_numpy(u).to("cuda")
        b = torch.empty_like(a)
        bms = time_steps(lambda: jac.tblock(a, b, T, t=t, bx=bx, by=by, waves=w), args.steps, 1)
        del a, b
        torch.cuda.empty_cache()
        rows.append({"t": t, "tile_bx_by": [bx, by], "waves": w, "ms_per_step": round(ms, 3),
                     "glups": round(lups / (ms * 1e-3) / 1e9, 2),
                     "two_grid_tblock_glups": round(lups / (bms * 1e-3) / 1e9, 2),
                     "memory_gb": round(comp_bytes / 1e9, 3), "passes": math.ceil(T / t)})
        print(f"  t {t}: {rows[-1]['glups']} GLUP/s in one array, "
              f"{rows[-1]['two_grid_tblock_glups']} in two", file=sys.stderr, flush=True)
    best = max(rows, key=lambda r: r["glups"])
    achieved = 16 * N ** 3 / (best["ms_per_step"] / best["passes"] * 1e-3) / 1e9
    ms_copy = copy_bandwidth(jac)
    return {"metric": "GLUP/s, 512^3 FP64 Jacobi T=100, compressed single grid", "unit": "GLUP/s",
            "copy_bandwidth_gbs": round(ms_copy, 1),
            "value": best["glups"], "higher_is_better": True, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
            "dtype": "f64", "data": "synthetic: uniform [0,1) interior and shell, numpy default_rng(0)",
            "config": {"workload": "jacobi3d 512^3 interior, FP64, T=100, one array",
                       **{k: best[k] for k in ("t", "tile_bx_by", "waves", "passes")}},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": comp_traffic(best),
                         "traffic_unit": "GB per launch",
                         "note": "per pass incl. its plane copies and shell rewrite"},
            "memory_gb": {"compressed": best["memory_gb"],
                          "two_grids": round(2 * 514 ** 3 * 8 / 1e9, 3)},
            "by_depth": rows}


def comp_traffic(row):
    """HBM GB per pass of the compressed-grid kernel from its committed
    profile, when that profile measured this instance with the current sources."""
    bx, by = row["tile_bx_by"]
    inst = f"compressed_kernel<double, {row['t']}, {bx // 64}, {by // row['waves']}, {row['waves']}>"
    fig = profile_figures(f"compressed_f64_t{row['t']}_512cubed.md", inst)
    return fig.get("traffic_gb_per_launch") if fig else None


def bench_refine(args):
    """Laplace solve to a relative FP64 residual of 1e-10 from a zero interior:
    FP64 refinement around FP32 blocked inner sweeps (50 per outer iteration)
    against all-FP64 blocked Jacobi checked every 50 sweeps.  Both need the
    same number of sweeps (the inner sweeps from e = 0 reproduce the outer
    Jacobi iteration), which the spectral sweep count predicts exactly.
    --refine-outer K > 0 runs K outer iterations (50 K FP64 sweeps) instead
    of the full solves and projects the time to the tolerance."""
    import torch
    from paper_0912_4506_amd import inputs, perf_model
    from paper_0912_4506_amd import jacobi as jac
    from paper_0912_4506_amd.refine import refine_solve, jacobi_solve_f64

    n, tol, inner = args.refine_n, args.refine_tol, 50
    g = inputs.laplace_problem(n, n, n, seed=0)
    predicted = perf_model.jacobi_sweeps_to_tolerance(g, tol, check_every=inner)
    bounded = args.refine_outer > 0
    run_tol = 1e-300 if bounded else tol
    res = {"predicted_sweeps": predicted}
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    def timed(fn):
        x = torch.from_numpy(g).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn(x)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    if not args.skip_mixed:
        t = args.refine_t
        dt = jac.default_tile(g.shape, inner, t, dtype=torch.float32, rhs=True)
        (x, outer, rel), sec = timed(lambda x: refine_solve(
            x, tol=run_tol, inner=inner, t=t, check_every=args.check_every,
            max_outer=args.refine_outer if bounded else 10 ** 6,
            callback=lambda it, r: log(f"  mixed outer {it} rel {r:.3e}") if it % 2000 == 0 else None))
        del x
        sweeps = outer * inner
        res["mixed"] = {"inner_tile": {"t": dt[0], "bx": dt[1], "by": dt[2], "waves": dt[4]},
                        "seconds": round(sec, 2), "outer": outer, "sweeps": sweeps,
                        "rel_residual": rel, "ms_per_50_sweeps": round(1e3 * sec / max(outer, 1), 3),
                        "projected_seconds": round(sec * predicted / max(sweeps, 1), 1)}
        log(json.dumps({"mixed": res["mixed"]}))
    if not args.skip_f64:
        # the all-FP64 reference runs at the autotuner's choice for this grid
        # and check interval (cached by the library for the solve's calls)
        xa = torch.from_numpy(g).to("cuda")
        (tt, tbx, tby, tw), _ = jac.autotune(xa, torch.empty_like(xa), inner * args.check_every,
                                             reps=1)
        del xa
        torch.cuda.empty_cache()
        dt = (tt, tbx, tby, 0, tw)
        (x, sweeps, rel), sec = timed(lambda x: jacobi_solve_f64(
            x, tol=run_tol, check=inner * args.check_every,
            max_sweeps=inner * args.refine_outer if bounded else 10 ** 9,
            callback=lambda s, r: log(f"  f64 sweeps {s} rel {r:.3e}") if s % 100000 == 0 else None))
        del x
        res["fp64"] = {"tile": {"t": dt[0], "bx": dt[1], "by": dt[2], "waves": dt[4]},
                       "seconds": round(sec, 2), "sweeps": sweeps, "rel_residual": rel,
                       "ms_per_50_sweeps": round(1e3 * sec * inner / max(sweeps, 1), 3),
                       "projected_seconds": round(sec * predicted / max(sweeps, 1), 1)}
        log(json.dumps({"fp64": res["fp64"]}))
    # the dominant kernel: the inner FP32 sweeps with a right-hand side, alone
    # (algorithmic traffic 12 B per cell and pass: e in and out, r in)
    ea = torch.zeros(g.shape, dtype=torch.float32, device="cuda")
    eb = torch.zeros_like(ea)
    r32 = torch.rand(g.shape, dtype=torch.float32, device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(0))
    ims = time_steps(lambda: jac.tblock(ea, eb, inner, t=args.refine_t, rhs=r32), 5, 1)
    it = jac.default_tile(g.shape, inner, args.refine_t, dtype=torch.float32, rhs=True)[0]
    ipasses = math.ceil(inner / it)
    iach = 12 * n ** 3 * ipasses / (ims * 1e-3) / 1e9
    res["inner_solve"] = {"ms": round(ims, 3), "t": it, "passes": ipasses,
                          "glups": round(n ** 3 * inner / (ims * 1e-3) / 1e9, 1),
                          "achieved_gbs": round(iach, 1)}
    del ea, eb, r32
    torch.cuda.empty_cache()
    # HBM traffic of that kernel from its committed profile (rocprofv3
    # FETCH_SIZE/WRITE_SIZE scaled by the copy kernel's), while the kernel
    # sources and the default blocking are those it was measured on
    res["copy_bandwidth_gbs"] = round(copy_bandwidth(jac), 1)
    # (the passes' depths differ by at most one: the profile covers the
    # depth most of them run at)
    _, ibx, iby, _, iw = jac.default_tile(g.shape, inner, args.refine_t, dtype=torch.float32, rhs=True)
    idepth = dominant_depth(inner, ipasses)
    fig = profile_figures(f"refine_{n}cubed.md",
                          f"tblock_kernel<float, {idepth}, {ibx // 64}, {iby // iw}, {iw}, 1>")
    key = "projected_seconds" if bounded else "seconds"
    out = {"metric": f"Laplace solve {n}^3 to {tol:g} relative FP64 residual "
                     + ("(projected from a bounded run)" if bounded else "(wall clock)"),
           "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "dtype": "f32 inner sweeps, f64 residual and update",
           "config": {"workload": f"Laplace {n}^3, tol {tol:g}, {inner} inner sweeps per outer step"},
           "data": "synthetic: uniform [0,1) Dirichlet data, zero initial interior",
           "roofline": {"bound": "hbm", "kernel": "the inner FP32 blocked pass with a right-hand side",
                        "achieved": round(iach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(iach / HBM_PEAK_GBS, 4),
                        "traffic": fig.get("traffic_gb_per_launch") if fig else None,
                        "traffic_unit": f"GB per launch (the depth-{idepth} passes)",
                        "algorithmic_bytes_per_launch": 12 * n ** 3},
           "results": res}
    if "mixed" in res:
        out["value"] = res["mixed"][key]
        if "fp64" in res:
            out["speedup_vs_fp64"] = round(res["fp64"][key] / res["mixed"][key], 3)
    return out


def bench_fp32(args):
    """The blocked pass in FP32: 512^3, T = 100 (8 B per cell and pass) and
    the refinement's inner form, 768^3, T = 50 with a right-hand side (12 B
    per cell and pass), each at the library's default blocking of every depth
    2..8 and at its default depth.  The input is the FP64 workload's seeded
    grid cast to FP32; the right-hand side is uniform [0, 1)."""
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    f32 = torch.float32

    def sweep(n, T, rhs, bytes_per_cell):
        a = torch.from_numpy(inputs.grid(n, n, n, seed=0)).to("cuda", f32)
        b = torch.empty_like(a)
        r = (torch.rand(a.shape, dtype=f32, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(0)) if rhs else None)
        rows = {}
        for t in range(2, 9):
            tt, bx, by, _, w = jac.default_tile(a.shape, T, t, dtype=f32, rhs=rhs)
            try:
                ms = time_steps(lambda: jac.tblock(a, b, T, t=tt, bx=bx, by=by, waves=w, rhs=r),
                                args.steps, args.warmup)
            except Exception as e:                # a depth the menu cannot run
                rows[str(t)] = f"refused: {e}"
                continue
            passes = math.ceil(T / tt)
            rows[str(t)] = {"glups": round(n ** 3 * T / (ms * 1e-3) / 1e9, 1), "tile": [bx, by],
                            "waves": w, "passes": passes,
                            "achieved_gbs": round(bytes_per_cell * n ** 3 * passes / (ms * 1e-3) / 1e9, 1)}
        d = jac.default_tile(a.shape, T, 0, dtype=f32, rhs=rhs)
        del a, b, r
        torch.cuda.empty_cache()
        return rows, d

    rows, d = sweep(512, 100, False, 8)
    best = rows[str(d[0])]
    rrows, rd = sweep(768, 50, True, 12)
    return {"metric": "GLUP/s, 512^3 FP32 Jacobi T=100, temporal-blocked", "value": best["glups"],
            "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "dtype": "f32",
            "data": "synthetic: the FP64 workload's uniform [0,1) grid cast to FP32",
            "config": {"workload": "jacobi3d 512^3 interior, FP32, T=100", "t": d[0],
                       "tile_bx_by": [d[1], d[2]], "waves": d[4]},
            "roofline": {"bound": "hbm", "achieved": best["achieved_gbs"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(best["achieved_gbs"] / HBM_PEAK_GBS, 4),
                         "traffic": None, "algorithmic_bytes_per_launch": 8 * 512 ** 3},
            "by_depth": rows,
            "rhs_768": {"T": 50, "default_t": rd[0], "by_depth": rrows}}


def bench_lbm(args):
    """D3Q19 lattice Boltzmann (BGK, periodic 256^3 box, omega = 1.7): the
    fused pull stream-collide kernel (one step per pass) and the depth-2
    temporally blocked pass (two steps per pass), FP64 and FP32, against the
    HBM roofline (19 populations read and written per pass)."""
    import torch
    from paper_0912_4506_amd import inputs, jacobi as jac

    n, T = args.lbm_n, args.lbm_steps
    T += T % 2                                     # whole two-step passes
    cells = n ** 3
    res = {}
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        f = torch.from_numpy(inputs.lbm_populations(n, n, n, seed=0)).to("cuda", dt)
        g = torch.empty_like(f)
        state = {"f": f, "g": g}
        res[name] = {}
        runs = [("plain", False, 1, 0)] + [("t2", True, 2, int(k)) for k in args.lbm_kchunks.split(",")]
        if ("t2", True, 2, 0) not in runs:
            runs.append(("t2", True, 2, 0))
        for method, blocked, per_pass, kchunk in runs:
            def step(blocked=blocked, kchunk=kchunk):
                out = jac.lbm_d3q19(state["f"], state["g"], 1.7, T, blocked=blocked, kchunk=kchunk)
                if out is state["g"]:
                    state["f"], state["g"] = state["g"], state["f"]

            ms = time_steps(step, args.steps, args.warmup)
            bpl = 2 * 19 * f.element_size() / per_pass     # algorithmic bytes per update
            lups = cells * T / (ms * 1e-3)
            achieved = lups * bpl / 1e9
            row = {"glups": round(lups / 1e9, 3), "ms_per_step": round(ms, 3),
                   "kernel_ms": round(ms / (T // per_pass), 4),
                   "bytes_per_lup": bpl, "achieved_gbs": round(achieved, 1),
                   "frac": round(achieved / HBM_PEAK_GBS, 4)}
            if method == "t2":
                row["kchunk"] = kchunk or "library"
                res[name].setdefault("t2_by_kchunk", []).append(row)
                if kchunk:
                    continue
            res[name][method] = row
        res[name]["t2"]["vs_plain"] = round(res[name]["t2"]["glups"] / res[name]["plain"]["glups"], 3)
        del f, g, state
        torch.cuda.empty_cache()
    ms_copy = copy_bandwidth(jac)
    for r in res.values():
        for m in [r["plain"], r["t2"]] + r["t2_by_kchunk"]:
            m["frac_of_copy"] = round(m["achieved_gbs"] / ms_copy, 4)
    best = max(("plain", "t2"), key=lambda m: res["f64"][m]["glups"])
    f64 = res["f64"][best]
    return {"metric": f"GLUP/s, D3Q19 lattice Boltzmann {n}^3 periodic box, BGK", "unit": "GLUP/s",
            "value": f64["glups"], "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f64["ms_per_step"], "dtype": "f64",
            "data": "synthetic: populations (1 + 0.1 U[0,1)) / 19, numpy default_rng(0)",
            "config": {"workload": f"D3Q19 BGK {n}^3, omega 1.7, {T} steps per step",
                       "method": {"plain": "one step per pass, 64x4 blocks",
                                  "t2": "two steps per pass, 32x8 regions, 30x6 output tiles (FP32: 32x16)"}[best]},
            "roofline": {"bound": "hbm", "achieved": f64["achieved_gbs"], "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": f64["frac"], "traffic": None,
                         "algorithmic_bytes_per_lup": f64["bytes_per_lup"]},
            "by_dtype": res, "copy_bandwidth_gbs": round(ms_copy, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="metric",
                    choices=["metric", "batched", "adjoint", "refine", "pipelined", "compressed", "lbm",
                             "fp32"])
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the blocking first")
    ap.add_argument("--tmax", type=int, default=8, help="deepest blocking depth the autotuner tries")
    ap.add_argument("--t", type=int, default=0, help="pin the blocking depth (skips autotuning)")
    ap.add_argument("--bx", type=int, default=0, help="pin the block shape (with --t)")
    ap.add_argument("--by", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--depths", default="1,2,3,4,5,6,8,16",
                    help="depths reported in by_depth (best block shape each)")
    ap.add_argument("--traffic", default=None,
                    help="measured HBM GB per blocked launch to report as roofline.traffic")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--noncubic", action="store_true")
    ap.add_argument("--relaxed-only", action="store_true",
                    help="batched: time the relaxed graph replay only (no lockstep or per-grid runs)")
    ap.add_argument("--refine-n", type=int, default=768)
    ap.add_argument("--refine-tol", type=float, default=1e-10)
    ap.add_argument("--refine-t", type=int, default=0,
                    help="inner FP32 sweeps per pass (0: the library's choice)")
    ap.add_argument("--refine-outer", type=int, default=0,
                    help="> 0: bounded run of that many outer iterations, time projected")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--check-every", type=int, default=1)
    ap.add_argument("--skip-f64", action="store_true")
    ap.add_argument("--lbm-n", type=int, default=256)
    ap.add_argument("--lbm-steps", type=int, default=20)
    ap.add_argument("--lbm-kchunks", default="4,8,12,16,64",
                    help="z chunks timed for the depth-2 pass (the library default always runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    ensure_built()
    fn = {"metric": bench_metric, "batched": bench_batched, "adjoint": bench_adjoint,
          "refine": bench_refine, "pipelined": bench_pipelined,
          "compressed": bench_compressed, "lbm": bench_lbm, "fp32": bench_fp32}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
