"""Benchmark: steady-state NRxx solve of the lid-driven cavity on one MI355X.

A step is one full solve (Alg. 2 V-cycles + mass correction + stop test,
Sec. 3.2.3) from the global Maxwellian to the workload's tolerance, on the
128x128 lid-driven cavity (Shakhov Pr 2/3, Kn 0.075, M = 5, second-order
minmod, lid 0.5, 4-level V-cycle, tol 1e-10).  `value` is the whole-job
smoother throughput: cell-moment updates made by fast-sweeping steps inside
the timed region divided by the timed wall time.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "smoother cell-moment updates/s + time-to-residual 1e-8, plain vs mixed/learned"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2206_13164_amd", "csrc", f)
               for f in ("nrxx_device.hpp", "nrxx_kernels.hip", "nrxx_batch.hip")]
PROFILES = os.path.join(ROOT, "profiles")
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def per_update_cost(M: int, order: int, coarse: bool, fp_bytes: int = 8):
    """Algorithmic cost of one cell update of the smoother (estimate of the
    method, independent of the kernel): bytes = read + write of the cell
    record (+ the right-hand-side record on coarse levels); flops = 3 C(M+4,4)
    FMA per basis change times the number of changes (4 faces + normalise at
    first order, 8 face states + normalise at second order, + 1 for the
    right-hand side on coarse levels) plus ~80 flops per coefficient."""
    N = math.comb(M + 3, 3)
    P = (5 if order == 1 else 9) + (1 if coarse else 0)
    flops = 2 * P * 3 * math.comb(M + 4, 4) + 80 * N
    nbytes = 2 * (N + 3) * fp_bytes + ((N + 3) * fp_bytes if coarse else 0)
    return flops, nbytes


def cycle_accounting(spec):
    """Cell updates, launches, flops and bytes of the smoother in one V-cycle."""
    L = spec["levels"]
    tot = dict(cells=0, launches=0, flops=0.0, bytes=0.0)
    for k in range(L):
        nx, ny = spec["nx"] >> k, spec["ny"] >> k
        steps = spec["s3"] if k == L - 1 else spec["s1"] + spec["s2"]
        fl, by = per_update_cost(spec["M"], spec["order"], coarse=k > 0)
        cells = steps * 4 * nx * ny
        tot["cells"] += cells
        tot["launches"] += steps * 4 * (nx + ny - 1)
        tot["flops"] += cells * fl
        tot["bytes"] += cells * by
    return tot


def kernel_source_hash() -> str:
    """sha256 over the code of the sweep kernels' sources (comments and
    whitespace removed, so that editing a comment does not invalidate a
    committed counter summary)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        text = open(f).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when the summary is missing or
    was taken on a different kernel source."""
    import hashlib
    path = os.path.join(PROFILES, f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    src = kernel_source_hash()
    if vals.get("kernel_source_sha256") != src or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(spec, seconds_hint: float):
    """The oracle (FP64, serial paper-order sweeps, one thread) on a bounded
    sample: one V-cycle of the same workload from the Maxwellian start."""
    import oracle
    from paper_2206_13164_amd import inputs as I
    oracle.set_threads(1)
    P = oracle.problem(spec)
    st = I.maxwellian_state(spec)
    acc = cycle_accounting(spec)
    t0 = time.perf_counter()
    oracle.vcycle(P, st)
    dt = time.perf_counter() - t0
    N = math.comb(spec["M"] + 3, 3)
    return {"value": acc["cells"] * N / dt, "unit": "cell-moment updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one V-cycle ({acc['cells']} cell updates) of the same workload from the "
                      f"Maxwellian start, serial Gauss-Seidel order, 1 thread, {dt:.1f} s"}


def time_variant(spec, tol, max_cycles, ref, NA):
    """One warm-up and one timed solve of a variant of the workload (same
    start, same stopping rule): time-to-residual and cycle count."""
    import torch
    from paper_2206_13164_amd import nrxx as N
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ctx.solve(st, tol, max_cycles, ref_norm=ref)
    ctx.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, cyc, hist = ctx.solve(st, tol, max_cycles, ref_norm=ref)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc != N.NRXX_OK:
        raise SystemExit(f"variant did not converge: rc={rc} cycles={cyc} last={hist[-1]:.3e}")
    ms, cells, _ = ctx.sweep_stats(reset=True)
    ctx.close()
    return {"precision": "fp32 sweeps + fp64 defect correction" if spec.get("precision") else "fp64",
            "time_to_residual_s": wall, "cycles": cyc, "final_rel_residual": hist[-1] / ref}


def learned_leg(max_cycles):
    """Config-5 comparison on a held-out cavity (256x256, M = 5, 6 levels,
    tol 1e-8 relative to the Maxwellian start's residual): plain FP64 from
    the Maxwellian vs the learned start in FP64 and with FP32 smoothing
    blocks; times include the network's inference and the start check."""
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import warmstart as W
    if not os.path.exists(W.DEFAULT_WEIGHTS):
        return {"skipped": "no trained network"}
    ws = W.WarmStart()
    s = I.cavity_draws(1, I.SEED_TEST, sides=(256,), Ms=(5,), levels=6)[0]
    r = W.compare(s, ws, tol=1e-8, max_cycles=max_cycles)
    base = r["maxwellian_p0"]["seconds"]
    return {"cavity": {"grid": "256x256", "M": 5, "Kn": s["Kn"], "lid": s["wall_u"][2],
                       "collision": "Shakhov" if s["collision"] else "BGK", "levels": 6,
                       "tol": 1e-8},
            **r,
            "speedup_learned_fp64": base / r["learned_p0"]["seconds"],
            "speedup_learned_mixed": base / r["learned_p1"]["seconds"],
            "network": {k: v for k, v in ws.meta.items() if k != "loss"}}


def baselines_leg(spec, max_cycles):
    """The paper's comparison of solvers (Sec. 2.4, 3.1, 3.2) on the first-order
    version of the workload: the NMG solve to the workload's tolerance, then
    explicit time marching (forward Euler, global step) and single-level fast
    sweeping from the same Maxwellian start for the same wall time, each with
    the relative residual it reaches and its cell-update rate.  Forward Euler
    with the unlimited central slopes of the second-order workload itself
    turns non-physical; the steps it survives there are reported too."""
    import torch
    from paper_2206_13164_amd import nrxx as N
    NA = math.comb(spec["M"] + 3, 3)
    cells = spec["nx"] * spec["ny"]
    s1 = dict(spec, order=1)
    ctx = N.Context(s1)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)
    ctx.solve(st, spec["tol"], max_cycles, ref_norm=ref)
    ctx.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, cyc, hist = ctx.solve(st, spec["tol"], max_cycles, ref_norm=ref)
    torch.cuda.synchronize()
    budget = time.perf_counter() - t0
    out = {"workload": "first-order version of the benchmark cavity", "budget_s": budget,
           "nmg": {"cycles": cyc, "seconds": budget, "rel_residual": hist[-1] / ref,
                   "converged": rc == N.NRXX_OK}}

    def march(c, st, step, chunk):
        c.init_maxwellian(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget:
            step(st, chunk)
            n += chunk
        torch.cuda.synchronize()
        return n, time.perf_counter() - t0

    ctx.euler(st, nsteps=10)  # load the code objects
    n, wall = march(ctx, st, lambda x, k: ctx.euler(x, nsteps=k), 200)
    out["euler"] = {"steps": n, "seconds": wall, "rel_residual": ctx.residual(st) / ref,
                    "cell_moment_updates_per_s": n * cells * NA / wall}
    ctx.close()
    ctx = N.Context(dict(s1, levels=1))
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ctx.sweep(st, nsteps=1)
    def fs_steps(x, k):
        ctx.sweep(x, nsteps=k)
        torch.cuda.synchronize()  # sweeps are asynchronous: keep the clock honest

    n, wall = march(ctx, st, fs_steps, 4)
    out["fast_sweeping_single_level"] = {
        "steps": n, "seconds": wall, "rel_residual": ctx.residual(st) / ref,
        "cell_moment_updates_per_s": 4 * n * cells * NA / wall}
    ctx.close()
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    n = 0
    try:
        while n < 20000:
            ctx.euler(st, nsteps=100)
            n += 100
        out["euler_second_order_central"] = {"steps": n, "non_physical": False}
    except N.NrxxError:
        out["euler_second_order_central"] = {"steps_before_non_physical": n, "non_physical": True}
    ctx.close()
    return out


def four_sided_leg(max_cycles):
    """The paper's solver table for the four-sided cavity (Sec. 4.2, 64x64,
    M = 5, Shakhov, Kn 0.777): iterations and wall time to the relative
    residual 1e-8 of forward Euler (steps of the global step), single-level
    fast sweeping (four-direction steps, each followed by the mass
    correction) and NMG (V-cycles), all from the global Maxwellian.  The
    paper's CPU figures are quoted beside them as context."""
    import torch
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import nrxx as N
    s = I.spec("four_sided64_shakhov_m5")
    tol = s["tol"]
    out = {"workload": "four_sided64_shakhov_m5", "tol": tol,
           "paper_cpu": {"iterations": {"euler": 4442, "fast_sweeping": 607, "nmg": 17},
                         "seconds": {"euler": 6031.19, "fast_sweeping": 2068.4, "nmg": 295.75}}}

    def timed_solve(spec):
        ctx = N.Context(spec)
        st = ctx.empty(0)
        ctx.init_maxwellian(st)
        ref = ctx.residual(st)
        ctx.solve(st, tol, 2, ref_norm=ref)  # load the code objects
        ctx.init_maxwellian(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, cyc, hist = ctx.solve(st, tol, max_cycles, ref_norm=ref)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.close()
        return {"iterations": cyc, "seconds": wall, "converged": rc == N.NRXX_OK,
                "rel_residual": hist[-1] / ref}

    out["nmg"] = timed_solve(s)
    out["fast_sweeping"] = timed_solve(dict(s, levels=1, s3=1))
    ctx = N.Context(s)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)
    ctx.euler(st, nsteps=2)
    ctx.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, r = 0, ref
    while r > tol * ref and n < 20000:
        ctx.euler(st, nsteps=1)
        n += 1
        r = ctx.residual(st)
    wall = time.perf_counter() - t0
    ctx.close()
    out["euler"] = {"iterations": n, "seconds": wall, "converged": r <= tol * ref,
                    "rel_residual": r / ref}
    return out


def batch_leg(n=16, cycles=6):
    """Batched throughput: n drawn cavities (sides 64/96/128, M 3/5/8,
    BGK/Shakhov, Kn log-uniform in [0.01, 1]) in one batch after autotuning,
    `cycles` graph-replayed V-cycles."""
    import torch
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import nrxx as N
    specs = I.cavity_draws(n, I.SEED_BATCH, sides=(64, 96, 128))
    b = N.Batch(specs)
    st = b.empty_states()
    b.init_maxwellian(st)
    b.autotune(st)
    b.solve(st, 0.0, 1)  # capture the graphs, load the code objects
    b.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, cyc, nrm, ref = b.solve(st, 0.0, cycles, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = sum(int(c) * cycle_accounting(x)["cells"] * math.comb(x["M"] + 3, 3) for c, x in zip(cyc, specs))
    tun = [b.tuning(g) for g in range(b.groups())]
    b.close()
    return {"problems": n, "cycles": cycles, "seconds": wall,
            "cell_moment_updates_per_s": upd / wall,
            "tuning": [{k: t[k] for k in ("M", "order", "problems", "team_width", "grid", "unit_order")}
                       for t in tun]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lid128_shakhov_m5_central")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start comparison (256x256 held-out cavity)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-throughput leg")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the explicit-Euler and single-level fast-sweeping comparison")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-sweep (precision 1) solve of the same workload")
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--schedule", type=int, default=0,
                    help="sweep schedule: 0 automatic (= 3), 1 per-diagonal launches, "
                         "2 static persistent, 3 work queue with overlapping sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver's "
              "multi-GPU decomposition is a design, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import nrxx as N

    if args.copy_bytes:
        # plain copy of a known size: reads and writes copy_bytes each
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes}))
        return

    spec = I.spec(args.workload, schedule=args.schedule)
    tol = spec["tol"]
    M = spec["M"]
    NA = math.comb(M + 3, 3)
    torch.cuda.set_device(0)
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)

    def one_solve():
        ctx.init_maxwellian(st)
        rc, cyc, hist = ctx.solve(st, tol, args.max_cycles, ref_norm=ref)
        return rc, cyc, hist

    for _ in range(args.warmup):
        one_solve()
    ctx.sweep_stats(reset=True)
    sched = ctx.level_schedule(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = []
    for _ in range(args.steps):
        rc, cyc, hist = one_solve()
        cycles.append(cyc)
        if rc != N.NRXX_OK:
            raise SystemExit(f"solve did not converge: rc={rc} cycles={cyc} last={hist[-1]:.3e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, sweep_cells, launches = ctx.sweep_stats(reset=True)
    wall = t1 - t0
    acc = cycle_accounting(spec)
    ncyc = sum(cycles)
    assert abs(sweep_cells - ncyc * acc["cells"]) < 0.5, (sweep_cells, ncyc * acc["cells"])
    value = sweep_cells * NA / wall
    avg_launch_s = sweep_ms * 1e-3 / launches
    flops_per_launch = ncyc * acc["flops"] / launches
    bytes_per_launch = ncyc * acc["bytes"] / launches
    achieved_tflops = flops_per_launch / avg_launch_s / 1e12
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    kname = {3: "k_bsweep", 2: "k_sweep_persist"}.get(sched, "k_sweep_diag")
    traffic = profiled_traffic(kname, args.workload)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-moment updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": f"{spec['nx']}x{spec['ny']}", "M": M, "N_alpha": NA,
            "collision": "Shakhov" if spec["collision"] else "BGK", "Kn": spec["Kn"],
            "order": spec["order"], "limiter": "minmod" if spec["limiter"] == 0 else "central",
            "levels": spec["levels"], "tol": tol, "start": "global Maxwellian",
        },
        "time_to_residual_s": wall / args.steps,
        "cycles_per_solve": cycles,
        "sweep_kernel_rate": sweep_cells * NA / (sweep_ms * 1e-3),
        "sweep_share_of_wall": sweep_ms * 1e-3 / wall,
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "kernel": kname + {3: " (work queue: up to 8 overlapping directional sweeps of one level per "
                                  "launch)",
                               2: " (static persistent: up to 16 directional sweeps of one level per launch)"}
                              .get(sched, " (one anti-diagonal of one sweep direction per launch)"),
            "launches": launches,
            "avg_launch_us": avg_launch_s * 1e6,
            "flops_per_launch": flops_per_launch,
            "bytes_per_launch": bytes_per_launch,
            "hbm_achieved_GBs": achieved_gbs,
            "hbm_frac": achieved_gbs / PEAK_HBM_GBS,
        },
    }
    if not args.no_mixed:
        out["mixed"] = time_variant(dict(spec, precision=1), tol, args.max_cycles, ref, NA)
        out["mixed"]["speedup_vs_plain"] = (wall / args.steps) / out["mixed"]["time_to_residual_s"]
    if not args.no_baselines:
        out["baselines"] = baselines_leg(spec, args.max_cycles)
        out["baselines"]["four_sided_64"] = four_sided_leg(args.max_cycles * 5)
    if not args.no_batch:
        out["batch"] = batch_leg()
    if not args.no_learned:
        out["learned"] = learned_leg(args.max_cycles)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, 20.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
