"""Summarise a rocprofv3 kernel trace over the timed window of a bench run.

bench.py prints the host clock bracket of its timed region to stderr as

    [bench] timed window monotonic_ns <start> <end> boottime_ns <start> <end>

and rocprofv3 (``--kernel-trace``, SQLite output) stamps every dispatch on
the same monotonic clock.  This tool keeps the dispatches that lie inside
the window and prints, per kernel, the launch count, total and average
duration and the launch shape, plus the share of the window during which
any kernel ran.

    python -m paper_2206_13164_amd.profsum trace TRACE_results.db BENCH_STDERR
    python -m paper_2206_13164_amd.profsum counters PMC_results.db [BENCH_STDERR]

The second form sums each counter over its hardware instances per dispatch
(``--pmc`` runs) and prints the per-dispatch average per kernel, over the
timed window when the bench's stderr is given.  The single-problem legs log
their solves as ``<label> window monotonic_ns <start> <end>`` (label = the
workload, plus ``_fp64`` / ``_fp32_blocks`` on the heated cavity);
``--window LABEL`` selects one of those instead of the headline's.
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3


def window(stderr_text: str, label: str = "timed"):
    """Host-clock window the bench logged as '<label> window monotonic_ns a b'."""
    m = re.search(re.escape(label) + r" window monotonic_ns (\d+) (\d+)", stderr_text)
    if not m:
        raise SystemExit(f"no '{label} window' line in the bench output")
    return int(m.group(1)), int(m.group(2))


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("nrxx::", "")
    return re.sub(r"\(.*", "", name)


def summarise(db: str, w0: int, w1: int):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, duration, grid_x, workgroup_x, vgpr_count, "
                       "lds_size, scratch_size from kernels").fetchall()
    per = collections.OrderedDict()
    spans = []
    for name, s, e, d, gx, wx, vgpr, lds, scr in rows:
        if s < w0 or e > w1:
            continue
        k = short_name(name)
        t = per.setdefault(k, dict(calls=0, ns=0, shape=None))
        t["calls"] += 1
        t["ns"] += d
        t["shape"] = dict(workgroups=gx // max(wx, 1), threads=wx, vgpr=vgpr, lds=lds, scratch=scr)
        spans.append((s, e))
    spans.sort()
    busy, cs, ce = 0, None, None
    for s, e in spans:
        if cs is None or s > ce:
            if cs is not None:
                busy += ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    if cs is not None:
        busy += ce - cs
    return per, busy


def counters(db: str, w0=None, w1=None):
    """{kernel: {counter: (dispatches, mean per dispatch)}} from a --pmc run."""
    con = sqlite3.connect(db)
    q = ("select name, dispatch_id, counter_name, sum(counter_value), min(start), max(end) "
         "from pmc_events group by name, dispatch_id, counter_name")
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, disp, cname, val, s, e in con.execute(q):
        if w0 is not None and (s < w0 or e > w1):
            continue
        acc[short_name(name)][cname].append(val)
    return {k: {c: (len(v), sum(v) / len(v)) for c, v in d.items()} for k, d in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters"])
    ap.add_argument("db")
    ap.add_argument("bench_stderr", nargs="?")
    ap.add_argument("--window", default="timed",
                    help="label of the logged window (default: the headline's timed window)")
    args = ap.parse_args()
    if args.mode == "counters":
        w = window(open(args.bench_stderr).read(), args.window) if args.bench_stderr else (None, None)
        res = counters(args.db, *w)
        names = sorted({c for d in res.values() for c in d})
        print("| kernel | dispatches | " + " | ".join(names) + " |")
        print("|---|---:|" + "---:|" * len(names))
        for k, d in sorted(res.items()):
            n = max(v[0] for v in d.values())
            print(f"| `{k}` | {n} | " + " | ".join(f"{d[c][1]:.6g}" if c in d else "" for c in names) + " |")
        return
    if not args.bench_stderr:
        raise SystemExit("trace mode needs the bench's stderr")
    w0, w1 = window(open(args.bench_stderr).read(), args.window)
    per, busy = summarise(args.db, w0, w1)
    W = w1 - w0
    print(f"{args.window} window {W / 1e6:.1f} ms; some kernel running {busy / 1e6:.1f} ms "
          f"({100.0 * busy / max(W, 1):.0f} %)")
    print(f"| kernel | calls | total ms | avg us | workgroups x threads, VGPRs, LDS B, scratch B |")
    print("|---|---:|---:|---:|---|")
    for k, t in sorted(per.items(), key=lambda kv: -kv[1]["ns"]):
        sh = t["shape"]
        print(f"| `{k}` | {t['calls']} | {t['ns'] / 1e6:.1f} | {t['ns'] / t['calls'] / 1e3:.1f} | "
              f"{sh['workgroups']} x {sh['threads']}, {sh['vgpr']}, {sh['lds']}, {sh['scratch']} |")


if __name__ == "__main__":
    main()
