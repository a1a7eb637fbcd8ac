"""Benchmark of the NRxx steady-state solver (FAS V-cycles over fast-sweeping
smoothers, Alg. 1-2 of the paper) on one MI355X.  Prints one JSON line.

Headline workload: 64 lid-driven cavities drawn from rng(220613164) (side
uniform in {64, 96, 128, 192, 256}, Kn log-uniform in [0.01, 1], lid speed
uniform in [0.1, 0.5], M uniform in {3, 5, 8}, BGK or Shakhov at 50/50,
second order with central slopes, walls at theta 1, levels down to an 8- or
12-cell coarsest grid), solved together as one batch: autotuned sweep
schedule, one graph-captured NMG iteration per group of equal (M, order).
A step is one NMG iteration (V-cycle, mass correction, residual norm, stop
test) of all 64 cavities.  `value` = smoother cell-moment updates made in
the timed steps / timed wall time.  `time_to_residual_s` = one solve of the
whole batch from the global Maxwellian until every cavity has reached the
relative residual 1e-8.

Legs beside the headline: the bottom-heated 256x256 M = 8 cavity at
Kn 0.05 and 0.2 in FP64 and with FP32 smoothing blocks (mirror symmetry,
field difference), held-out 256x256 M = 5 cavities from the Maxwellian and
from the learned warm start, the single 128x128 M = 5 cavity, and the FP64
oracle on the host cores (one thread in the serial order and all threads in
the anti-diagonal order, plus a whole 32x32 M = 3 solve).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "smoother cell-moment updates/s + time-to-residual 1e-8, plain vs mixed/learned"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2206_13164_amd", "csrc", f)
               for f in ("nrxx_device.hpp", "nrxx_kernels.hip", "nrxx_batch.hip", "nrxx_wave.hpp",
                         "nrxx_wsweep.hip")]
PROFILES = os.path.join(ROOT, "profiles")
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
HEADLINE = "batch64_lid_mixed"  # the 64 drawn cavities


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    """Cell updates, flops, bytes and dependent anti-diagonal steps of the
    smoother in one V-cycle (gamma = 1)."""
    L = spec["levels"]
    tot = dict(cells=0, flops=0.0, bytes=0.0, chain=0)
    for k in range(L):
        nx, ny = spec["nx"] >> k, spec["ny"] >> k
        steps = spec["s3"] if k == L - 1 else spec["s1"] + spec["s2"]
        fl, by = per_update_cost(spec["M"], spec["order"], coarse=k > 0)
        cells = steps * 4 * nx * ny
        tot["cells"] += cells
        tot["flops"] += cells * fl
        tot["bytes"] += cells * by
        tot["chain"] += steps * 4 * (nx + ny - 1)
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


def sweep_traffic(workload: str):
    """{kernel symbol: HBM bytes per launch} of the batch's sweep kernels
    from the committed FETCH_SIZE / WRITE_SIZE summary, or None when it is
    missing or was taken on a different kernel source."""
    path = os.path.join(PROFILES, f"sweep_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    out, sha = {}, None
    for line in open(path):
        if line.startswith("- kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip().strip("`")
        m = line.strip().split("|")
        if len(m) > 6 and m[1].strip().startswith("`k_"):
            try:
                out[m[1].strip().strip("`")] = float(m[-2])
            except ValueError:
                pass
    if sha != kernel_source_hash() or not out:
        return None
    return out


def host_cpu():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


# ---------------------------------------------------------------------------
# Headline: the 64-cavity batch
# ---------------------------------------------------------------------------

def time_to_residual(b, st, max_cycles):
    """The whole batch from the Maxwellian until every cavity has reached
    the relative residual 1e-8 (graph-replayed cycles); closes the batch."""
    import torch
    b.set_timing(False)
    b.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, cyc, nrm, ref = b.solve(st, 1e-8, max_cycles, use_graph=True)
    torch.cuda.synchronize()
    ttr = time.perf_counter() - t0
    log(f"time to residual {ttr:.1f} s")
    b.close()
    return ttr, cyc, nrm, ref, rc


def apply_tuning(b, tunings):
    """Set every group's sweep tuning from a list written by --tuning-out
    (matched by (M, order))."""
    by = {(t["M"], t["order"]): t for t in tunings}
    for g in range(b.groups()):
        cur = b.tuning(g)
        t = by[(cur["M"], cur["order"])]
        b.set_tuning(g, t["team_width"], t["grid"], t["unit_order"], t["split"], kernel=t["kernel"],
                     rows_per_sync=t["rows_per_sync"])


def sweep_kernel_name(t):
    """Kernel symbol (template arguments as rocprofv3 prints them) of a
    group's sweep tuning."""
    if t["kernel"] == 1:
        return f"k_wsweep<{t['M']}, {t['order']}, {2 if t['M'] >= 7 else 4}>"
    return (f"k_bsweep<double, {t['M']}, {t['order']}, {t['team_width']}, "
            f"{'true' if t['split'] else 'false'}>")


def headline(args):
    import torch
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import nrxx as N
    specs = I.cavity_draws(64, I.SEED_BATCH)
    NA = [math.comb(s["M"] + 3, 3) for s in specs]
    acc = [cycle_accounting(s) for s in specs]
    b = N.Batch(specs)
    st = b.empty_states()
    b.init_maxwellian(st)
    t0 = time.perf_counter()
    if args.tuning_in:
        apply_tuning(b, json.load(open(args.tuning_in)))
    else:
        b.autotune(st)
    tune_s = time.perf_counter() - t0
    log(f"autotune {tune_s:.1f} s" if not args.tuning_in else f"tuning read from {args.tuning_in}")
    if args.tuning_out:
        with open(args.tuning_out, "w") as fh:
            json.dump([b.tuning(g) for g in range(b.groups())], fh)
    b.set_timing(True)
    b.init_maxwellian(st)
    b.solve(st, 0.0, max(1, args.warmup), use_graph=False)  # warm-up cycles
    for g in range(b.groups()):
        b.kernel_stats(g, reset=True)
    torch.cuda.synchronize()
    w0 = (time.monotonic_ns(), time.clock_gettime_ns(time.CLOCK_BOOTTIME))
    t0 = time.perf_counter()
    # eagerly enqueued cycles: HIP events around every sweep launch (events
    # recorded by graph nodes report no elapsed time); the time-to-residual
    # solve below replays the captured graphs
    rc, cyc, nrm, ref = b.solve(st, 0.0, args.steps, use_graph=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    w1 = (time.monotonic_ns(), time.clock_gettime_ns(time.CLOCK_BOOTTIME))
    # the timed window on the host clocks, to select its dispatches in a trace
    log(f"timed window monotonic_ns {w0[0]} {w1[0]} boottime_ns {w0[1]} {w1[1]}")
    assert all(int(c) == args.steps for c in cyc), cyc
    upd = sum(args.steps * a["cells"] * n for a, n in zip(acc, NA))
    # sweep kernels over the timed steps (HIP events on each group's stream)
    groups, tot_ms, tot_launch, tot_flops, tot_bytes = [], 0.0, 0.0, 0.0, 0.0
    for g in range(b.groups()):
        t = b.tuning(g)
        ms, nl, cf, cc = b.kernel_stats(g)
        ff, bf = per_update_cost(t["M"], t["order"], coarse=False)
        fc, bc = per_update_cost(t["M"], t["order"], coarse=True)
        fl, by = cf * ff + cc * fc, cf * bf + cc * bc
        tot_ms += ms
        tot_launch += nl
        tot_flops += fl
        tot_bytes += by
        groups.append({"M": t["M"], "order": t["order"], "problems": t["problems"],
                       "kernel": sweep_kernel_name(t),
                       "team_width": t["team_width"], "grid": t["grid"], "unit_order": t["unit_order"],
                       "split": t["split"], "launches": nl, "avg_launch_us": ms * 1e3 / max(nl, 1),
                       "cell_updates": cf + cc, "achieved_tflops": fl / max(ms, 1e-30) / 1e9,
                       "hbm_GBs": by / max(ms, 1e-30) / 1e6})
    log(f"timed {args.steps} cycles in {wall:.2f} s")
    if args.no_ttr:
        b.close()
        ttr, cyc2, nrm2, ref2, rc2 = float("nan"), [0], [0.0], [1.0], -1
    else:
        ttr, cyc2, nrm2, ref2, rc2 = time_to_residual(b, st, args.max_cycles)
    achieved = tot_flops / max(tot_ms, 1e-30) / 1e9  # TFLOP/s per launch-second
    # HBM bytes per launch from the committed counter summary, when it was
    # taken on these kernels (same source, same per-group kernels)
    tb = sweep_traffic(HEADLINE)
    traffic = None
    if tb is not None and all(g["kernel"] in tb for g in groups):
        traffic = sum(g["launches"] * tb[g["kernel"]] for g in groups) / max(tot_launch, 1)
    # critical path: the longest chain of dependent cell updates of one
    # cavity in a cycle (anti-diagonal steps of every directional sweep)
    chains = [(a["chain"], s) for a, s in zip(acc, specs)]
    chain, big = max(chains, key=lambda x: x[0])
    cyc_ms = wall / args.steps * 1e3

    gbs = tot_bytes / max(tot_ms, 1e-30) / 1e6
    conv = [bool(nrm2[i] <= 1e-8 * ref2[i]) for i in range(len(nrm2))]
    upd2 = sum(int(c) * a["cells"] * n for c, a, n in zip(cyc2, acc, NA))
    out = {
        "value": upd / wall,
        "ms_per_step": wall / args.steps * 1e3,
        "config": {
            "workload": HEADLINE,
            "problems": len(specs), "seed": I.SEED_BATCH,
            "sides": sorted({s["nx"] for s in specs}), "M": sorted({s["M"] for s in specs}),
            "Kn_range": [min(s["Kn"] for s in specs), max(s["Kn"] for s in specs)],
            "order": 2, "limiter": "central", "collision": "BGK/Shakhov (Pr 2/3)",
            "cell_values": sum(s["nx"] * s["ny"] * (n + 3) for s, n in zip(specs, NA)),
            "step": "one NMG iteration (V-cycle + mass correction + norm + stop test) of all 64 "
                    "cavities, enqueued eagerly with a HIP event pair around every sweep launch",
            "start": "global Maxwellian",
        },
        "time_to_residual_s": ttr,
        "time_to_residual": {"tol": 1e-8, "all_converged": all(conv) and rc2 == N.NRXX_OK,
                             "measured": not args.no_ttr,
                             "cycles_min": int(min(cyc2)), "cycles_mean": float(sum(cyc2)) / len(cyc2),
                             "cycles_max": int(max(cyc2)), "cell_moment_updates_per_s": upd2 / ttr,
                             "autotune_s": tune_s},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "limiter": "latency of the dependent cell updates, not FP64 issue or HBM bandwidth",
            "hbm_target": {"frac_wanted": 0.5, "frac": gbs / PEAK_HBM_GBS,
                           "met": gbs / PEAK_HBM_GBS >= 0.5,
                           "shortfall_x": 0.5 / max(gbs / PEAK_HBM_GBS, 1e-30)},
            "critical_path": {
                "cavity": f"{big['nx']}x{big['ny']}, M = {big['M']}, {big['levels']} levels",
                "dependent_updates_per_cycle": chain,
                "cycle_ms": cyc_ms,
                "us_per_dependent_update_if_chain_bound": cyc_ms * 1e3 / chain,
                "note": "a cycle can not finish before this chain of dependent cell updates of "
                        "its largest cavity; us_per_dependent_update_if_chain_bound is the time "
                        "per link at which the measured cycle would be the chain alone",
            },
            "kernel": "batched work-queue sweep kernels (k_wsweep: one wavefront per cell, or "
                      "k_bsweep: cell teams, per group as autotuned; up to 8 directional sweeps "
                      "of one level per launch)",
            "launches": tot_launch,
            "avg_launch_us": tot_ms * 1e3 / max(tot_launch, 1),
            "flops_per_launch": tot_flops / max(tot_launch, 1),
            "bytes_per_launch": tot_bytes / max(tot_launch, 1),
            "hbm_achieved_GBs": gbs,
            # the groups' launches overlap in time, so dividing each launch's
            # work by its own duration understates what the device does as a
            # whole; this is all groups' sweep work over the timed wall time
            "timed_window": {"achieved": tot_flops / max(wall * 1e3, 1e-30) / 1e9,
                             "frac": tot_flops / max(wall * 1e3, 1e-30) / 1e9 / PEAK_FP64_TFLOPS,
                             "hbm_GBs": tot_bytes / max(wall * 1e3, 1e-30) / 1e6,
                             "note": "sweep flops and algorithmic bytes of all groups over the "
                                     "timed wall time (device-level rate of the concurrent groups)"},
            "hbm_frac": gbs / PEAK_HBM_GBS,
            "note": "groups of different M run concurrently on their own streams, so their launch "
                    "durations overlap; flops per launch are the algorithmic estimate per cell "
                    "update times the updates of that launch",
            "groups": groups,
        },
    }
    return out


# ---------------------------------------------------------------------------
# Legs
# ---------------------------------------------------------------------------

def mirror_x(rec, M):
    """The x-mirror image of a state: cells i -> nx-1-i, u1 -> -u1 and
    coefficients with odd alpha_1 change sign."""
    from paper_2206_13164_amd import inputs as I
    import numpy as np
    al = I.alpha_list(M)
    m = rec[:, ::-1, :].copy()
    m[..., 0] = -m[..., 0]
    odd = al[:, 0] % 2 == 1
    m[..., 3:][..., odd] *= -1.0
    return m


def state_err(a, b, M):
    import numpy as np
    from paper_2206_13164_amd import inputs as I
    n = I.alpha_list(M).sum(axis=1)
    rho, th = b[..., 3], b[..., 2]
    eu = (np.abs(a[..., :2] - b[..., :2]).max(axis=-1) / np.sqrt(th)).max()
    et = (np.abs(a[..., 2] - b[..., 2]) / th).max()
    ef = (np.abs(a[..., 3:] - b[..., 3:]) / (rho[..., None] * th[..., None] ** (n / 2.0))).max()
    return float(max(eu, et, ef))


def solve_timed(spec, tol, max_cycles, ref=None, label=None):
    """One warm-up cycle, then a timed solve from the Maxwellian; returns the
    record, the final host state and the context's sweep statistics.  With a
    label, the solve's window on the host clock is logged under it (for
    selecting its dispatches in a kernel trace)."""
    import torch
    from paper_2206_13164_amd import nrxx as N
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    if ref is None:
        ref = ctx.residual(st)
    ctx.solve(st, 0.0, 1)
    ctx.init_maxwellian(st)
    ctx.sweep_stats(reset=True)
    torch.cuda.synchronize()
    w0 = time.monotonic_ns()
    t0 = time.perf_counter()
    rc, cyc, hist = ctx.solve(st, tol, max_cycles, ref_norm=ref)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if label:
        log(f"{label} window monotonic_ns {w0} {time.monotonic_ns()}")
    sms, scells, slaunch = ctx.sweep_stats(reset=True)
    host = ctx.to_host(st, math.comb(spec["M"] + 3, 3) + 3)
    ctx.close()
    acc = cycle_accounting(spec)
    rec = {"precision": "fp32 smoothing blocks + fp64 defect correction" if spec.get("precision")
           else "fp64", "seconds": wall, "cycles": cyc, "converged": rc == N.NRXX_OK,
           "final_rel_residual": hist[-1] / ref,
           "critical_path": {"dependent_steps_per_cycle": acc["chain"],
                             "ms_per_cycle": wall / max(cyc, 1) * 1e3,
                             "us_per_dependent_step": wall / max(cyc, 1) / acc["chain"] * 1e6},
           "sweep_kernel": {"launches": slaunch, "avg_launch_us": sms * 1e3 / max(slaunch, 1),
                            "share_of_wall": sms * 1e-3 / wall}}
    return rec, host, ref


def heated_leg(max_cycles):
    """The bottom-heated 256x256 cavity (Shakhov, M = 8, central slopes,
    5 levels) at Kn 0.05 and 0.2: FP64 and FP32-block solves to 1e-8, the
    x-mirror asymmetry of the converged FP64 field and the difference between
    the two converged fields."""
    from paper_2206_13164_amd import inputs as I
    out = {}
    for name in ("heated256_shakhov_m8_kn005", "heated256_shakhov_m8_kn02"):
        s = I.spec(name)
        p0, h0, ref = solve_timed(s, s["tol"], max_cycles, label=f"{name}_fp64")
        p1, h1, _ = solve_timed(dict(s, precision=1), s["tol"], max_cycles, ref=ref,
                                label=f"{name}_fp32_blocks")
        out[name] = {"Kn": s["Kn"], "fp64": p0, "fp32_blocks": p1,
                     "speedup_fp32_blocks": p0["seconds"] / p1["seconds"],
                     "mirror_asymmetry_fp64": state_err(mirror_x(h0, 8), h0, 8),
                     "mirror_asymmetry_fp32_blocks": state_err(mirror_x(h1, 8), h1, 8),
                     "fp32_blocks_vs_fp64_field": state_err(h1, h0, 8)}
        log(f"{name}: fp64 {p0['seconds']:.2f} s, fp32 blocks {p1['seconds']:.2f} s")
    return out


def learned_leg(draws, max_cycles):
    """Held-out 256x256 M = 5 cavities (rng(220613166)): plain FP64 from the
    Maxwellian against the learned start in FP64 and with FP32 smoothing
    blocks, each to 1e-8 relative to the Maxwellian start's residual; the
    learned times include the network's inference and the start check."""
    from paper_2206_13164_amd import inputs as I
    from paper_2206_13164_amd import warmstart as W
    if not os.path.exists(W.DEFAULT_WEIGHTS):
        return {"skipped": "no trained network"}
    ws = W.WarmStart()
    rows = []
    for s in I.cavity_draws(draws, I.SEED_TEST, sides=(256,), Ms=(5,), levels=6):
        r = W.compare(s, ws, tol=1e-8, max_cycles=max_cycles)
        base = r["maxwellian_p0"]["seconds"]
        rows.append({"Kn": s["Kn"], "lid": s["wall_u"][2],
                     "collision": "Shakhov" if s["collision"] else "BGK", **r,
                     "speedup_learned_fp64": base / r["learned_p0"]["seconds"],
                     "speedup_learned_fp32_blocks": base / r["learned_p1"]["seconds"]})
        log(f"learned draw Kn {s['Kn']:.3f}: {base:.2f} s -> {r['learned_p1']['seconds']:.2f} s")
    tot0 = sum(r["maxwellian_p0"]["seconds"] for r in rows)
    tot1 = sum(r["learned_p1"]["seconds"] for r in rows)
    return {"grid": "256x256", "M": 5, "levels": 6, "tol": 1e-8, "draws": rows,
            "total_seconds_maxwellian_fp64": tot0, "total_seconds_learned_fp32_blocks": tot1,
            "speedup_total": tot0 / tot1,
            "network": {k: v for k, v in ws.meta.items() if k not in ("loss", "validation")}}


def single_leg(workload, max_cycles):
    """One cavity alone (latency-bound: one cell team per cell on the
    dependency chain of the sweeps)."""
    from paper_2206_13164_amd import inputs as I
    s = I.spec(workload)
    rec, _, _ = solve_timed(s, s["tol"], max_cycles, label=workload)
    NA = math.comb(s["M"] + 3, 3)
    rec["workload"] = workload
    rec["cell_moment_updates_per_s"] = rec["cycles"] * cycle_accounting(s)["cells"] * NA / rec["seconds"]
    return rec


def cpu_baseline():
    """The FP64 oracle on the host: one V-cycle of the first drawn cavity of
    the batch (64x64, M = 8, BGK, 4 levels) from the Maxwellian, once in the
    serial order on one thread and once in the anti-diagonal order on every
    usable core (bitwise the same result), plus a whole solve of the
    32x32 M = 3 BGK cavity to 1e-8 on every core."""
    import numpy as np
    import oracle
    from paper_2206_13164_amd import inputs as I
    model, ncpu, usable = host_cpu()
    s = I.cavity_draws(1, I.SEED_BATCH)[0]
    NA = math.comb(s["M"] + 3, 3)
    cells = cycle_accounting(s)["cells"]
    P = oracle.problem(s)
    res = {}
    for mode, threads in (("serial_1_thread", 1), ("antidiagonal_all_cores", usable)):
        oracle.set_threads(threads)
        oracle.set_vcycle_wavefront(threads > 1)
        st = I.maxwellian_state(s)
        t0 = time.perf_counter()
        oracle.vcycle(P, st)
        dt = time.perf_counter() - t0
        res[mode] = {"threads": threads, "seconds": dt, "cell_moment_updates_per_s": cells * NA / dt}
        res.setdefault("_states", []).append(st)
    same = bool(np.array_equal(*res.pop("_states")))
    c1 = I.spec("lid32_bgk_m3")
    P1 = oracle.problem(c1)
    st = I.maxwellian_state(c1)
    t0 = time.perf_counter()
    rc, cyc, hist = oracle.solve(P1, st, c1["tol"], 200)
    c1_s = time.perf_counter() - t0
    oracle.set_vcycle_wavefront(False)
    oracle.set_threads(1)
    best = res["antidiagonal_all_cores"]
    return {"value": best["cell_moment_updates_per_s"], "unit": "cell-moment updates/s",
            "cores": usable, "kind": "oracle",
            "sample": f"one V-cycle ({cells} cell updates, N_alpha {NA}) of the batch's first cavity "
                      f"(64x64, M = 8, BGK, Kn {s['Kn']:.3f}, 4 levels) from the Maxwellian, "
                      f"anti-diagonal order on {usable} threads ({best['seconds']:.1f} s)",
            "cpu_model": model, "nproc": ncpu, "usable_cores": usable, **res,
            "parallel_equals_serial": same,
            "lid32_bgk_m3_time_to_residual": {"seconds": c1_s, "cycles": cyc, "threads": usable,
                                              "converged": rc == 0}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed NMG iterations of the batch")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-cycles", type=int, default=400)
    ap.add_argument("--legs", default="heated,learned,single,cpu",
                    help="comma list of heated, learned, single, cpu (or 'none')")
    ap.add_argument("--learned-draws", type=int, default=4)
    ap.add_argument("--no-ttr", action="store_true",
                    help="skip the batch's time-to-residual solve (profiling runs)")
    ap.add_argument("--single-workload", default="lid128_shakhov_m5_central")
    ap.add_argument("--tuning-out", default=None, help="write the groups' sweep tunings (JSON)")
    ap.add_argument("--tuning-in", default=None,
                    help="take the groups' sweep tunings from a --tuning-out file instead of autotuning")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver's "
              "multi-GPU decomposition is a design, not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes}))
        return
    torch.cuda.set_device(0)
    legs = set() if args.legs == "none" else set(args.legs.split(","))
    h = headline(args)
    out = {"metric": METRIC, "value": h.pop("value"), "unit": "cell-moment updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": h.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", **h}
    if "heated" in legs:
        out["heated256_m8"] = heated_leg(args.max_cycles)
    if "learned" in legs:
        out["learned"] = learned_leg(args.learned_draws, args.max_cycles)
    if "single" in legs:
        out["single_cavity"] = single_leg(args.single_workload, args.max_cycles)
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
