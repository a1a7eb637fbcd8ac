"""Reproduce the paper's solver tables on the GPU: iterations and wall time
to the relative residual 1e-8 of forward Euler (global step), single-level
fast sweeping (four-direction steps, each followed by the mass correction)
and the NMG solver, all from the global Maxwellian, for the cavity setups of
Sec. 4 (single lid-driven, Tables 1 and 2; M = 10, Table 3; the ES-BGK
model, Table 4;
four-sided, Table 6; bottom-heated, Table 8; second order, Table 9).  The iteration counts belong to the
method and can be compared with the paper's; wall times are this GPU's.

    python -m paper_2206_13164_amd.paper_tables [--min-side 0] [--max-side 128] [--tables 3,4]
        [--nmg-only] [--out FILE]

Prints one JSON line per row.
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import inputs as I
from . import nrxx as N

U_W = 0.2097  # 50 m/s at 273 K in units of sqrt(R T0)

# (table, label, spec overrides, paper iterations (Euler, FS, NMG))
ROWS = [
    ("1", "single lid, Kn 0.1, 32x32", dict(Kn=0.1, nx=32), (1823, 231, 12)),
    ("1", "single lid, Kn 0.1, 64x64", dict(Kn=0.1, nx=64), (4100, 507, 12)),
    ("1", "single lid, Kn 0.1, 128x128", dict(Kn=0.1, nx=128), (8398, 1084, 13)),
    ("1", "single lid, Kn 0.1, 256x256", dict(Kn=0.1, nx=256), (16364, 2000, 14)),
    ("2", "single lid, Kn 1.0, 32x32", dict(Kn=1.0, nx=32), (1978, 277, 15)),
    ("2", "single lid, Kn 1.0, 64x64", dict(Kn=1.0, nx=64), (4952, 681, 18)),
    ("2", "single lid, Kn 1.0, 128x128", dict(Kn=1.0, nx=128), (11120, 1509, 21)),
    ("2", "single lid, Kn 1.0, 256x256", dict(Kn=1.0, nx=256), (24266, 3300, 27)),
    ("3", "single lid, Kn 0.1, M = 10, 64x64", dict(Kn=0.1, nx=64, M=10), (5244, 708, 17)),
    ("3", "single lid, Kn 1.0, M = 10, 64x64", dict(Kn=1.0, nx=64, M=10), (6051, 866, 23)),
    ("4", "single lid, ES-BGK, Kn 0.1, 64x64", dict(Kn=0.1, nx=64, collision=2, beta=2.0 / 3.0),
     (4085, 503, 12)),
    ("4", "single lid, ES-BGK, Kn 1.0, 64x64", dict(Kn=1.0, nx=64, collision=2, beta=2.0 / 3.0),
     (5053, 690, 19)),
    ("4", "single lid, ES-BGK, Kn 0.1, M = 10, 64x64",
     dict(Kn=0.1, nx=64, M=10, collision=2, beta=2.0 / 3.0), (5177, 700, 17)),
    ("4", "single lid, ES-BGK, Kn 1.0, M = 10, 64x64",
     dict(Kn=1.0, nx=64, M=10, collision=2, beta=2.0 / 3.0), (7663, 1105, 27)),
    ("6", "four-sided lid, Kn 0.777, 64x64", dict(Kn=0.777, nx=64, wall_u=[-U_W, U_W, U_W, -U_W]),
     (4442, 607, 17)),
    ("8", "bottom-heated, Kn 0.3, 64x64", dict(Kn=0.3, nx=64, wall_u=[0.0, 0.0, 0.0, 0.0],
                                               wall_theta=[2.0, 1.0, 1.0, 1.0]), (4073, 499, 13)),
    ("9", "single lid, Kn 0.1, 2nd order, 32x32", dict(Kn=0.1, nx=32, order=2), (None, 384, 18)),
    ("9", "single lid, Kn 0.1, 2nd order, 64x64", dict(Kn=0.1, nx=64, order=2), (None, 728, 17)),
    ("9", "single lid, Kn 0.1, 2nd order, 128x128", dict(Kn=0.1, nx=128, order=2), (None, 1331, 24)),
]


def row_spec(kw: dict) -> dict:
    """Shakhov, M = 5, first order unless stated (second order: the paper's
    central slopes; ES-BGK rows: collision 2 with beta = Pr as Sec. 4
    states), lid speed U_W on the top wall, coarsest grid 8x8."""
    n = kw["nx"]
    d = dict(M=5, collision=1, Pr=2.0 / 3.0, order=1, limiter=1, wall_u=[0.0, 0.0, U_W, 0.0],
             ny=n, levels=int(math.log2(n // 8)) + 1, tol=1e-8)
    d.update(kw)
    return I.spec(None, **d)


def solver_run(spec, max_cycles):
    import torch
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)
    ctx.solve(st, spec["tol"], 1, ref_norm=ref)  # load the code objects
    ctx.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, cyc, hist = ctx.solve(st, spec["tol"], max_cycles, ref_norm=ref)
    torch.cuda.synchronize()
    out = {"iterations": cyc, "seconds": time.perf_counter() - t0, "converged": rc == N.NRXX_OK}
    ctx.close()
    return out


def euler_run(spec, max_steps):
    import torch
    ctx = N.Context(spec)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)
    ctx.euler(st, nsteps=1)
    ctx.init_maxwellian(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, r = 0, ref
    try:
        while r > spec["tol"] * ref and n < max_steps:
            ctx.euler(st, nsteps=1)
            n += 1
            r = ctx.residual(st)
        out = {"iterations": n, "seconds": time.perf_counter() - t0, "converged": r <= spec["tol"] * ref}
    except N.NrxxError:
        out = {"iterations": n, "non_physical": True}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-side", type=int, default=128)
    ap.add_argument("--min-side", type=int, default=0)
    ap.add_argument("--tables", default=None, help="comma list of table numbers (default: all)")
    ap.add_argument("--nmg-only", action="store_true", help="skip the Euler and FS solvers")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    tables = set(args.tables.split(",")) if args.tables else None
    import torch
    torch.cuda.set_device(0)
    lines = []
    for table, label, kw, paper in ROWS:
        if kw["nx"] > args.max_side or kw["nx"] < args.min_side:
            continue
        if tables is not None and table not in tables:
            continue
        s = row_spec(kw)
        row = {"table": table, "case": label, "paper_iterations": dict(zip(("euler", "fs", "nmg"), paper))}
        row["nmg"] = solver_run(s, 200)
        if not args.nmg_only:
            row["fs"] = solver_run(dict(s, levels=1, s3=1), 20000)
        if paper[0] is not None and not args.nmg_only:
            row["euler"] = euler_run(s, 100000)
        lines.append(json.dumps(row))
        print(lines[-1], flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
