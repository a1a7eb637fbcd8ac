"""GPU: the warm-start network's kernels (BF16 MFMA products, FP32
accumulation, Adam) against the FP64 reference, and the fields <-> record
kernels against the reference closure."""
import numpy as np
import pytest

from gpu_common import context, require_gpu
from oracle import mlp as R
from paper_2206_13164_amd import inputs as I

pytestmark = pytest.mark.gpu


def bf16_round(a):
    """Round float64/float32 values to the nearest BF16 (ties to even), as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def setup(rows, seed=1):
    from paper_2206_13164_amd import nrxx as N
    rng = np.random.default_rng(seed)
    params = [(bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in I.mlp_init()]
    X = rng.normal(size=(rows, 8)).astype(np.float32)
    X[:, 0] = rng.uniform(-2, 0, size=rows)
    T = rng.normal(size=(rows, 9)).astype(np.float32)
    in_mean = X.mean(axis=0).astype(np.float32)
    in_std = (X.std(axis=0) + 0.5).astype(np.float32)
    out_mean = rng.normal(size=9).astype(np.float32)
    out_std = rng.uniform(0.5, 2.0, size=9).astype(np.float32)
    m = N.Mlp(I.MLP_LAYERS, max_rows=4096)
    m.set_params(params)
    m.set_scaling(in_mean, in_std, out_mean, out_std)
    Xs = (X.astype(np.float64) - in_mean) / in_std
    Ts = (T.astype(np.float64) - out_mean) / out_std
    return m, params, X, T, Xs, Ts, (in_mean, in_std, out_mean, out_std)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("rows", [37, 300, 4096])
def test_forward_matches_reference(rows):
    torch = require_gpu()
    m, params, X, T, Xs, Ts, sc = setup(rows)
    Y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = R.forward(params, bf16_round(Xs))
    want = want * sc[3] + sc[2]
    err = rel(Y, want)
    print(f"rows {rows}: forward relative error {err:.2e} (BF16 activations)")
    # BF16 rounding of the hidden activations: ~2^-9 per element, averaged
    # over 256-term products; measured 5e-5 to 8e-5
    assert err < 2e-3


def forward_bf16_operands(params, Xs):
    """The reference forward pass with every product's operands rounded to
    BF16 as the kernels feed them to the matrix cores (weights are BF16
    already): inputs and hidden activations rounded before each product,
    everything else FP64."""
    a = bf16_round(Xs)
    for k, (W, b) in enumerate(params):
        z = a @ W.T + b
        a = z if k == len(params) - 1 else bf16_round(R.silu(z))
    return a


@pytest.mark.parametrize("rows", [37, 4096])
def test_forward_elementwise_matches_bf16_operand_reference(rows):
    # element by element: what is left is FP32 accumulation order and the
    # rare BF16 rounding flip of a hidden activation that sits on a rounding
    # boundary (one BF16 ulp, 2^-8, in one term of a 256-term product)
    torch = require_gpu()
    m, params, X, T, Xs, Ts, sc = setup(rows, seed=7)
    Y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    want = forward_bf16_operands(params, Xs) * sc[3] + sc[2]
    # per output field, errors in units of that field's output scale
    e = np.abs(Y - want) / (np.abs(want) + sc[3])
    print(f"rows {rows}: element-wise error median {np.median(e):.2e}, 99.9% {np.quantile(e, 0.999):.2e}, "
          f"max {e.max():.2e}")
    assert np.median(e) < 1e-5
    assert e.max() < 2e-3


def test_gradients_match_reference():
    torch = require_gpu()
    m, params, X, T, Xs, Ts, _ = setup(1000, seed=2)
    g, loss = m.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    Y, cache = R.forward(params, bf16_round(Xs))
    grads = R.backward(params, cache, Y, Ts)
    assert abs(loss - R.loss(Y, Ts)) < 1e-2 * R.loss(Y, Ts)
    got = m.unflatten(g)
    for k, ((gW, gb), (wW, wb)) in enumerate(zip(got, grads)):
        eW, eb = rel(gW, wW), rel(gb, wb)
        print(f"layer {k}: dW rel {eW:.2e}, db rel {eb:.2e}")
        assert eW < 1e-2 and eb < 1e-2, k


def test_adam_step_matches_reference():
    # the optimiser kernel against the reference Adam fed the GPU's own
    # gradients (isolates the update from the BF16 products)
    torch = require_gpu()
    m, params, X, T, Xs, Ts, _ = setup(512, seed=3)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p0 = m.unflatten(m.get_params().astype(np.float64))
    g, _ = m.gradients(Xd, Td)
    gl = m.unflatten(g.astype(np.float64))
    zeros = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p0]
    want, _, _ = R.adam(p0, gl, zeros, zeros, 1, lr=1e-3)
    m.train_step(Xd, Td, 1e-3)
    got = m.unflatten(m.get_params().astype(np.float64))
    for (gW, gb), (wW, wb), (oW, ob) in zip(got, want, p0):
        assert np.allclose(gW - oW, wW - oW, rtol=1e-4, atol=1e-9)
        assert np.allclose(gb - ob, wb - ob, rtol=1e-4, atol=1e-9)


def test_training_reduces_loss():
    torch = require_gpu()
    m, params, X, T, Xs, Ts, sc = setup(2048, seed=4)
    # a smooth target the network can represent
    Tsm = np.stack([np.sin(X[:, 6] * 3) + X[:, 1], np.cos(X[:, 7] * 2), X[:, 0] * X[:, 6]] * 3,
                   axis=1).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(Tsm).cuda()
    l0 = m.train_step(Xd, Td, 1e-3, want_loss=True)
    for _ in range(300):
        m.train_step(Xd, Td, 1e-3)
    l1 = m.train_step(Xd, Td, 1e-3, want_loss=True)
    print(f"loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.1 * l0


@pytest.mark.parametrize("M", [3, 5, 8])
def test_fields_to_records_and_back(orc, M):
    torch = require_gpu()
    from paper_2206_13164_amd import nrxx as N
    s = I.spec(None, M=M, nx=16, ny=12, levels=1)
    ctx = context(s)
    rng = np.random.default_rng(M)
    F = np.zeros((6, 8, 9), dtype=np.float32)
    F[..., 0] = rng.uniform(0.5, 1.5, size=(6, 8))
    F[..., 1:3] = rng.uniform(-0.3, 0.3, size=(6, 8, 2))
    F[..., 3] = rng.uniform(0.7, 1.4, size=(6, 8))
    F[..., 4:] = rng.uniform(-0.05, 0.05, size=(6, 8, 5))
    st = ctx.empty(0)
    ctx.init_fields(st, torch.from_numpy(F).cuda())
    nrec = I.nalpha(M) + 3
    got = ctx.to_host(st, nrec)
    al = orc.alpha_list(M)
    for j in range(12):
        for i in range(16):
            want = R.fields_to_record(M, al, F[j // 2, i // 2].astype(np.float64))
            assert np.array_equal(got[j, i], want), (i, j)
    back = ctx.state_fields(st).cpu().numpy()
    assert np.allclose(back, np.repeat(np.repeat(F, 2, axis=0), 2, axis=1), rtol=1e-6, atol=1e-7)
    # a non-positive temperature is refused
    F[2, 3, 3] = -0.1
    with pytest.raises(N.NrxxError) as ei:
        ctx.init_fields(st, torch.from_numpy(F).cuda())
    assert ei.value.code == N.NRXX_ENONPHYS
