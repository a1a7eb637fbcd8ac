"""GPU: the learned warm start.  The committed network (trained on the GPU
by `python -m paper_2206_13164_amd.warmstart train` and gated by
`validate`) must never cost V-cycles on held-out cavities it never saw and
save some over them, and a broken prediction must fall back to the global
Maxwellian."""
import os

import numpy as np
import pytest

from gpu_common import context, require_gpu
from paper_2206_13164_amd import inputs as I

pytestmark = pytest.mark.gpu


def weights():
    from paper_2206_13164_amd import warmstart as W
    if not os.path.exists(W.DEFAULT_WEIGHTS):
        pytest.fail(f"trained network missing: {W.DEFAULT_WEIGHTS}")
    return W


def test_learned_start_never_costs_cycles_on_held_out_cavities():
    # held-out draws (a seed the training never used), 256x256, M = 5,
    # 6 levels, tol 1e-8 relative to the Maxwellian start's residual.  Per
    # draw: the learned start takes no more V-cycles than the Maxwellian
    # (at or above the validated Kn gate it is the Maxwellian), and the
    # learned start with FP32 blocks is not slower beyond timing noise (5 %);
    # over the draws it saves cycles
    require_gpu()
    W = weights()
    ws = W.WarmStart()
    assert ws.kn_gate is not None
    saved = []
    for s in I.cavity_draws(4, I.SEED_TEST, sides=(256,), Ms=(5,), levels=6):
        r = W.compare(s, ws, tol=1e-8, precision=(0, 1))
        m, l, lm = r["maxwellian_p0"], r["learned_p0"], r["learned_p1"]
        print(f"Kn {s['Kn']:.3f} lid {s['wall_u'][2]:.2f}: Maxwellian {m['cycles']} cycles "
              f"{m['seconds']:.2f} s; learned ({l['start']}, start norm {l['start_norm']:.2f}) "
              f"{l['cycles']} cycles {l['seconds']:.2f} s; learned + FP32 blocks {lm['cycles']} "
              f"cycles {lm['seconds']:.2f} s", flush=True)
        assert m["converged"] and l["converged"] and lm["converged"]
        assert l["cycles"] <= m["cycles"]
        assert lm["seconds"] <= 1.05 * m["seconds"]
        if s["Kn"] >= ws.kn_gate:
            assert l["start"] == "maxwellian"
        saved.append(m["cycles"] - l["cycles"])
    assert sum(saved) > 0


def test_fallback_to_maxwellian():
    torch = require_gpu()
    W = weights()
    ws = W.WarmStart(gate=False)  # the prediction path, whatever the draw's Kn
    s = I.cavity_draws(1, I.SEED_TEST, sides=(64,), Ms=(3,), levels=3)[0]
    ctx = context(s)
    st = ctx.empty(0)
    ctx.init_maxwellian(st)
    ref = ctx.residual(st)
    # a prediction with negative temperatures is refused
    z = np.load(W.DEFAULT_WEIGHTS, allow_pickle=False)
    out_mean = z["out_mean"].copy()
    out_mean[3] = -5.0
    ws.m.set_scaling(z["in_mean"], z["in_std"], out_mean, z["out_std"])
    used, n0 = ws.apply(ctx, st, s, ref)
    assert used == "maxwellian" and n0 == ref
    want = ctx.empty(0)
    ctx.init_maxwellian(want)
    assert bool((st == want).all())
    # a prediction worse than the Maxwellian is refused as well
    ws.m.set_scaling(z["in_mean"], z["in_std"], z["out_mean"] + 0.5, z["out_std"])
    used, _ = ws.apply(ctx, st, s, ref)
    assert used == "maxwellian"
    # at or above the Kn gate the prediction is not used
    wg = W.WarmStart()
    used, n0 = wg.apply(ctx, st, dict(s, Kn=max(s["Kn"], wg.kn_gate)), ref)
    assert used == "maxwellian" and n0 == ref


def test_training_data_generation_small():
    torch = require_gpu()
    from paper_2206_13164_amd import warmstart as W
    X, T, info = W.training_set(3, seed=11, chunk=2, log=lambda *_: None)
    assert X.shape == (3 * W.FIELD_GRID ** 2, 8) and T.shape == (3 * W.FIELD_GRID ** 2, 9)
    assert bool(torch.isfinite(T).all()) and bool((T[:, 0] > 0).all()) and bool((T[:, 3] > 0).all())
    assert all(x["used"] for x in info)
