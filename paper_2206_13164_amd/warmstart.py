"""Learned warm start: a network that maps cavity parameters and a position
to the macroscopic fields of the steady state, trained on steady states the
solver itself produces, and a solve that starts from its prediction with the
global Maxwellian as the fallback.

Every numerical step runs in the HIP library (batched solves, field
extraction, the network's forward/backward/Adam kernels, the fields-to-record
closure, residual norms); this module only assembles inputs, shuffles rows
and keeps the bookkeeping.

Command line (writes the weights file used by tests and the benchmark):
    python -m paper_2206_13164_amd.warmstart train --draws 2000 --out FILE
    python -m paper_2206_13164_amd.warmstart validate --draws 16
The second solves validation draws (never trained on) from the Maxwellian
and from the prediction and stores the Kn gate above which the prediction
is not used.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import inputs as I
from . import nrxx as N

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_mlp.npz")
FIELD_GRID = 64          # training fields: cavities solved on 64 x 64 cells
TRAIN_TOL = 1e-6         # their relative residual
TRAIN_LEVELS = 4


def field_grid(n: int) -> int:
    """Largest divisor of n not above FIELD_GRID (the network is evaluated on
    that grid and injected into the n-cell grid)."""
    for d in range(min(n, FIELD_GRID), 0, -1):
        if n % d == 0:
            return d
    return 1


class _FieldReader:
    """Per-M contexts used only to read fields of FIELD_GRID^2 states."""

    def __init__(self):
        self.ctx = {}

    def __call__(self, spec, state):
        M = spec["M"]
        if M not in self.ctx:
            self.ctx[M] = N.Context(I.spec(None, M=M, nx=spec["nx"], ny=spec["ny"], levels=1))
        return self.ctx[M].state_fields(state)


def training_set(n, seed=I.SEED_TRAIN, chunk=64, max_cycles=80, log=print):
    """Solve n drawn cavities on FIELD_GRID^2 cells to TRAIN_TOL with the
    batched solver; return input rows X (n_used * G^2 x 8), target rows T
    (x 9) as float32 CUDA tensors and per-draw records."""
    import torch
    draws = I.cavity_draws(n, seed, sides=(FIELD_GRID,), levels=TRAIN_LEVELS, tol=TRAIN_TOL)
    reader = _FieldReader()
    Xs, Ts, info = [], [], []
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        specs = draws[c0:c0 + chunk]
        b = N.Batch(specs)
        st = b.empty_states()
        b.init_maxwellian(st)
        try:
            rc, cyc, nrm, ref = b.solve(st, TRAIN_TOL, max_cycles)
            ok = [bool(np.isfinite(nrm[k]) and nrm[k] <= 1e-4 * ref[k]) for k in range(len(specs))]
        except N.NrxxError as e:  # one draw went non-physical: solve them one by one
            log(f"chunk {c0}: {e}; solving its draws one at a time")
            cyc, ok = [], []
            for k, s in enumerate(specs):
                ctx = N.Context(s)
                ctx.init_maxwellian(st[k])
                try:
                    r1, c1, h1 = ctx.solve(st[k], TRAIN_TOL, max_cycles)
                    ok.append(bool(h1[-1] <= 1e-4 * h1[0]))
                    cyc.append(c1)
                except N.NrxxError:
                    ok.append(False)
                    cyc.append(-1)
        for k, s in enumerate(specs):
            info.append(dict(Kn=s["Kn"], lid=s["wall_u"][2], M=s["M"], collision=s["collision"],
                             cycles=int(cyc[k]), used=ok[k]))
            if not ok[k]:
                continue
            F = reader(s, st[k]).reshape(-1, 9)
            Xs.append(torch.from_numpy(I.mlp_features(s, s["nx"], s["ny"])).cuda())
            Ts.append(F)
        b.close()
        log(f"draws {c0 + len(specs)}/{n}: {sum(x['used'] for x in info)} used, "
            f"{time.perf_counter() - t0:.1f} s")
    return torch.cat(Xs), torch.cat(Ts), info


def train(X, T, epochs=20, batch_rows=16384, lr=2e-3, lr_end=2e-5, seed=I.SEED_INIT, log=print):
    """Train the network on rows (X, T) with Adam and a cosine learning-rate
    decay; returns (Mlp, scaling, history)."""
    import torch
    rows = X.shape[0]
    in_mean = X.mean(dim=0).cpu().numpy()
    in_std = X.std(dim=0).cpu().numpy()
    in_std = np.where(in_std > 1e-6, in_std, 1.0).astype(np.float32)
    out_mean = T.mean(dim=0).cpu().numpy()
    out_std = T.std(dim=0).cpu().numpy()
    out_std = np.where(out_std > 1e-9, out_std, 1.0).astype(np.float32)
    m = N.Mlp(I.MLP_LAYERS, max_rows=batch_rows)
    m.set_params(I.mlp_init(seed))
    m.set_scaling(in_mean, in_std, out_mean, out_std)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    steps = epochs * max(1, rows // batch_rows)
    hist, step = [], 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(rows, device="cuda", generator=g)
        tot, nb = 0.0, 0
        for s0 in range(0, rows - batch_rows + 1, batch_rows):
            idx = perm[s0:s0 + batch_rows]
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
            lr_k = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * step / steps))
            want = (s0 // batch_rows) % 16 == 0
            loss = m.train_step(xb, tb, lr_k, want_loss=want)
            if want:
                tot += loss
                nb += 1
            step += 1
        hist.append(tot / max(nb, 1))
        log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return m, (in_mean, in_std, out_mean, out_std), hist


def save(path, m, scaling, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=m.get_params(), widths=np.array(m.widths, dtype=np.int32),
             in_mean=scaling[0], in_std=scaling[1], out_mean=scaling[2], out_std=scaling[3],
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


class WarmStart:
    """A trained network loaded into the library, and the warm-started
    initialisation with the Maxwellian fallback."""

    def __init__(self, path=DEFAULT_WEIGHTS, max_rows=FIELD_GRID * FIELD_GRID, gate=True):
        z = np.load(path, allow_pickle=False)
        self.m = N.Mlp([int(w) for w in z["widths"]], max_rows=max_rows)
        self.m.set_params(z["params"])
        self.m.set_scaling(z["in_mean"], z["in_std"], z["out_mean"], z["out_std"])
        self.meta = json.loads(bytes(z["meta"]).decode())
        # Kn from which the prediction is not used (set by `validate`): above
        # it the V-cycle's asymptotic rate, not the start, sets the cycles
        self.kn_gate = self.meta.get("kn_gate") if gate else None

    def fields(self, spec):
        """Predicted fields on the field grid of the cavity: (fny, fnx, 9)."""
        import torch
        fnx, fny = field_grid(spec["nx"]), field_grid(spec["ny"])
        X = torch.from_numpy(I.mlp_features(spec, fnx, fny)).cuda()
        return self.m.forward(X).reshape(fny, fnx, 9)

    def apply(self, ctx, state, spec, maxwellian_norm):
        """Fill `state` from the prediction; fall back to the global
        Maxwellian if Kn is at or above the validated gate, if the prediction
        is non-physical or if its residual norm is not below the
        Maxwellian's.  Returns (used, norm of the start)."""
        if self.kn_gate is not None and spec["Kn"] >= self.kn_gate:
            ctx.init_maxwellian(state)
            return "maxwellian", maxwellian_norm
        try:
            ctx.init_fields(state, self.fields(spec))
            nw = ctx.residual(state)
        except N.NrxxError:
            nw = float("inf")
        if math.isfinite(nw) and nw < maxwellian_norm:
            return "learned", nw
        ctx.init_maxwellian(state)
        return "maxwellian", maxwellian_norm


def compare(spec, ws, tol=1e-8, max_cycles=200, precision=(0, 1)):
    """Time-to-residual of the same cavity from the Maxwellian (FP64) and
    from the learned start (FP32 smoothing blocks when precision 1 is
    listed); the stop test uses ||R(Maxwellian)|| for both."""
    import torch
    out = {}
    for prec in precision:
        ctx = N.Context(dict(spec, precision=prec))
        st = ctx.empty(0)
        ctx.init_maxwellian(st)
        ref = ctx.residual(st)
        ctx.solve(st, 0.0, 1)  # warm the code objects
        for start in ("maxwellian", "learned"):
            if prec == 1 and start == "maxwellian":
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "learned":
                used, n0 = ws.apply(ctx, st, spec, ref)
            else:
                ctx.init_maxwellian(st)
                used, n0 = "maxwellian", ref
            rc, cyc, hist = ctx.solve(st, tol, max_cycles, ref_norm=ref)
            torch.cuda.synchronize()
            out[f"{start}_p{prec}"] = dict(start=used, cycles=cyc, seconds=time.perf_counter() - t0,
                                           converged=rc == N.NRXX_OK, start_norm=n0 / ref)
        ctx.close()
    return out


def validation_draws(n, after=2000, side=256, levels=6):
    """Draws after[..after+n] of the training stream (rng(SEED_TRAIN), the
    training set's draw order), never used in training, at side^2 cells and
    M = 5."""
    d = I.cavity_draws(after + n, I.SEED_TRAIN, sides=(FIELD_GRID,), levels=TRAIN_LEVELS,
                       tol=TRAIN_TOL)[after:]
    return [dict(s, nx=side, ny=side, M=5, levels=levels, tol=1e-8) for s in d]


def choose_gate(rows):
    """Smallest validation Kn at which the learned start saved no cycle
    (None when it saved cycles on every draw)."""
    bad = [r["Kn"] for r in rows if r["learned"] >= r["maxwellian"]]
    return min(bad) if bad else None


def validate(path, n, log=print):
    """Solve n validation draws from the Maxwellian and from the (ungated)
    prediction, choose the Kn gate and store it in the weights file."""
    ws = WarmStart(path, gate=False)
    rows = []
    for s in validation_draws(n):
        r = compare(s, ws, tol=1e-8, precision=(0,))
        rows.append(dict(Kn=s["Kn"], lid=s["wall_u"][2], maxwellian=r["maxwellian_p0"]["cycles"],
                         learned=r["learned_p0"]["cycles"]))
        log(json.dumps(rows[-1]))
    gate = choose_gate(rows)
    z = dict(np.load(path, allow_pickle=False))
    meta = json.loads(bytes(z["meta"]).decode())
    meta["kn_gate"] = gate
    meta["validation"] = rows
    z["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    np.savez(path, **z)
    log(json.dumps({"kn_gate": gate}))
    return gate, rows


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    v = sub.add_parser("validate")
    v.add_argument("--draws", type=int, default=16)
    v.add_argument("--weights", default=DEFAULT_WEIGHTS)
    t = sub.add_parser("train")
    t.add_argument("--draws", type=int, default=2000)
    t.add_argument("--epochs", type=int, default=20)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--eval", type=int, default=2, help="held-out draws to compare afterwards")
    t.add_argument("--eval-side", type=int, default=256)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    log = lambda s: print(s, flush=True)
    if args.cmd == "validate":
        validate(args.weights, args.draws, log=log)
        return
    t0 = time.perf_counter()
    X, T, info = training_set(args.draws, log=log)
    t1 = time.perf_counter()
    m, sc, hist = train(X, T, epochs=args.epochs, log=log)
    t2 = time.perf_counter()
    meta = dict(draws=args.draws, used=int(sum(x["used"] for x in info)), field_grid=FIELD_GRID,
                train_tol=TRAIN_TOL, epochs=args.epochs, loss=hist, seconds_data=t1 - t0,
                seconds_train=t2 - t1, seed_train=I.SEED_TRAIN, seed_init=I.SEED_INIT)
    save(args.out, m, sc, meta)
    log(json.dumps({k: v for k, v in meta.items() if k != "loss"}))
    if args.eval:
        ws = WarmStart(args.out)
        for s in I.cavity_draws(args.eval, I.SEED_TEST, sides=(args.eval_side,), Ms=(5,), levels=6):
            log(json.dumps(dict(Kn=s["Kn"], lid=s["wall_u"][2], **compare(s, ws))))


if __name__ == "__main__":
    main()
