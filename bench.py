"""Benchmark: 512^3 FP64 Jacobi, T = 100 sweeps, temporally blocked vs plain.

One step = T = 100 sweeps of the 512^3 (514^3 arrays) FP64 grid through
jacobi_tblock at the blocking depth t being measured; inputs are resident in
HBM before the timed region, and consecutive steps continue the iteration
(level 100 of one step is level 0 of the next; the work does not depend on
the values).  Prints ONE JSON line (rank 0, N = 1):

  value     GLUP/s of the blocked run at the reported depth (512^3 * 100 / time)
  roofline  the blocked kernel against HBM: algorithmic bytes per launch
            (16 B per cell per pass: one read and one write of each cell) over
            the kernel's average launch duration, measured with HIP events on
            the stream the kernels run on, against the 8 TB/s HBM peak
  plain     the plain sweep kernel under the same protocol
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
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

N = 512
T = 100
HBM_PEAK_GBS = 8000.0


def ensure_built():
    from paper_0912_4506_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def time_steps(fn, steps, warmup, stream):
    import torch
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
    """M_s: the library's copy kernel over two nbytes arrays (beyond the
    256 MB last-level cache), bytes read + written per second."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    ms = time_steps(lambda: jac.copy(dst, src), reps, 2, stream)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(u, target_s=12.0):
    """The CPU oracle (as it stands) on the host cores: whole 512^3 grid for
    as many sweeps as fit about target_s seconds."""
    import oracle
    t0 = time.perf_counter()
    oracle.sweeps(u, 1)
    t1 = time.perf_counter() - t0
    sweeps = max(1, min(T, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.sweeps(u, sweeps)
    dt = time.perf_counter() - t0
    return {"value": round(N ** 3 * sweeps / dt / 1e9, 4), "unit": "GLUP/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{N}^3 FP64 grid, {sweeps} of the {T} sweeps, one run ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--depths", default="1,2,4,5",
                    help="blocking depths to measure; the best one is reported")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    ensure_built()
    import numpy as np
    import torch

    from paper_0912_4506_amd import inputs, jacobi as jac

    u = inputs.grid(N, N, N, seed=0)
    a = torch.from_numpy(u).to("cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    lups = N ** 3 * T
    cell_bytes = 16 * N ** 3  # one read + one write of each cell per pass

    results = {}
    for t in [int(x) for x in args.depths.split(",") if x]:
        state = {"a": a, "b": b}

        def step(t=t, state=state):
            out = jac.tblock(state["a"], state["b"], T, t=t)
            if out is state["b"]:
                state["a"], state["b"] = state["b"], state["a"]

        ms = time_steps(step, args.steps, args.warmup, stream)
        passes = math.ceil(T / t)
        tile = jac.default_tile(a.shape, T, t)
        results[t] = {"ms_per_step": ms, "glups": lups / (ms * 1e-3) / 1e9, "passes": passes,
                      "kernel_ms": ms / passes, "tile": tile}
    best_t = max(results, key=lambda t: results[t]["glups"])
    best = results[best_t]

    plain = None
    if not args.no_plain:
        state = {"a": a, "b": b}

        def pstep(state=state):
            out = jac.plain(state["a"], state["b"], T)
            if out is state["b"]:
                state["a"], state["b"] = state["b"], state["a"]

        pms = time_steps(pstep, max(1, args.steps // 2), 1, stream)
        plain = {"glups": round(lups / (pms * 1e-3) / 1e9, 2), "ms_per_step": round(pms, 3),
                 "kernel_ms": round(pms / T, 4),
                 "hbm_gbs": round(cell_bytes / (pms / T * 1e-3) / 1e9, 1)}

    del a, b
    torch.cuda.empty_cache()
    ms_copy = copy_bandwidth(jac)

    achieved = cell_bytes / (best["kernel_ms"] * 1e-3) / 1e9
    line = {
        "metric": "GLUP/s & % roofline, 512³ FP64 Jacobi T=100: temporal-blocked vs plain",
        "value": round(best["glups"], 2),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(best["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: uniform [0,1) grid from numpy default_rng(0), interior and shell",
        "config": {"workload": f"jacobi3d {N}^3 interior (514^3 arrays) FP64, T={T}, Dirichlet shell",
                   "t": best_t, "tile_bx_by": best["tile"][1:3], "kchunk": best["tile"][3],
                   "passes": best["passes"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "plain": plain,
        "by_depth": {str(t): {"glups": round(r["glups"], 2), "kernel_ms": round(r["kernel_ms"], 4)}
                     for t, r in sorted(results.items())},
        "copy_bandwidth_gbs": round(ms_copy, 1),
        "roofline_p0_glups": round(ms_copy / 16, 2),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(u)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
