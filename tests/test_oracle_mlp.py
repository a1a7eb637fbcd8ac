"""Pins of the FP64 warm-start references (oracle/mlp.py): gradients against
central differences and against torch's autograd (an independent chain-rule
implementation), Adam's first step against its closed form, and the
fields -> record closure against quadrature moments of the distribution it
describes."""
import numpy as np
import pytest

import hermite_quad as HQ
from oracle import mlp as R
from paper_2206_13164_amd import inputs as I


def tiny(seed=0, layers=(3, 5, 4, 2)):
    rng = np.random.default_rng(seed)
    params = [(rng.normal(size=(layers[k + 1], layers[k])), rng.normal(size=layers[k + 1]))
              for k in range(len(layers) - 1)]
    X = rng.normal(size=(7, layers[0]))
    T = rng.normal(size=(7, layers[-1]))
    return params, X, T


def test_silu_closed_forms():
    assert R.silu(0.0) == 0.0 and R.silu_grad(0.0) == 0.5
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (R.silu(z + h) - R.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - R.silu_grad(z))) < 1e-8
    assert abs(R.silu(40.0) - 40.0) < 1e-12 and abs(R.silu(-40.0)) < 1e-12


def test_gradients_match_central_differences():
    params, X, T = tiny()
    Y, cache = R.forward(params, X)
    grads = R.backward(params, cache, Y, T)
    h = 1e-6
    for k, (W, b) in enumerate(params):
        for arr, g in ((W, grads[k][0]), (b, grads[k][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = R.loss(R.forward(params, X)[0], T)
                arr[idx] = old - h
                lm = R.loss(R.forward(params, X)[0], T)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.max(np.abs(fd - g)) <= 1e-6 * max(np.max(np.abs(g)), 1e-3), k


def test_gradients_match_torch_autograd():
    torch = pytest.importorskip("torch")
    params, X, T = tiny(seed=3, layers=(8, 16, 16, 9))
    Y, cache = R.forward(params, X)
    grads = R.backward(params, cache, Y, T)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    a = torch.tensor(X)
    for k, (W, b) in enumerate(tp):
        a = a @ W.T + b
        if k < len(tp) - 1:
            a = torch.nn.functional.silu(a)
    assert np.allclose(a.detach().numpy(), Y, rtol=1e-13, atol=1e-13)
    torch.mean((a - torch.tensor(T)) ** 2).backward()
    for (W, b), (gW, gb) in zip(tp, grads):
        assert np.allclose(W.grad.numpy(), gW, rtol=1e-12, atol=1e-14)
        assert np.allclose(b.grad.numpy(), gb, rtol=1e-12, atol=1e-14)


def test_adam_first_step_closed_form():
    # from m = v = 0, bias correction makes the first step -lr g / (|g| + eps)
    params, X, T = tiny(seed=5)
    Y, cache = R.forward(params, X)
    grads = R.backward(params, cache, Y, T)
    zeros = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    new, m, v = R.adam(params, grads, zeros, zeros, 1, lr=1e-2)
    for (W, b), (Wn, bn), (gW, gb) in zip(params, new, grads):
        assert np.allclose(Wn - W, -1e-2 * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=1e-15)
        assert np.allclose(bn - b, -1e-2 * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=1e-15)
    # and a few steps reduce the loss of a fixed batch
    p, mm, vv = params, zeros, zeros
    l0 = R.loss(Y, T)
    for t in range(1, 51):
        Yt, c = R.forward(p, X)
        g = R.backward(p, c, Yt, T)
        p, mm, vv = R.adam(p, g, mm, vv, t, lr=1e-2)
    assert R.loss(R.forward(p, X)[0], T) < 0.5 * l0


def test_default_initialisation_shapes_and_range():
    params = I.mlp_init()
    assert [W.shape for W, _ in params] == [(256, 8), (256, 256), (256, 256), (9, 256)]
    n = sum(W.size + b.size for W, b in params)
    assert n == 8 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 9 + 9
    for (W, b), fan in zip(params, I.MLP_LAYERS[:-1]):
        assert np.abs(W).max() <= 1 / np.sqrt(fan) and np.abs(b).max() <= 1 / np.sqrt(fan)


@pytest.mark.parametrize("M", [3, 5, 8])
def test_fields_to_record_moments_by_quadrature(orc, M):
    # the distribution described by the record has exactly the given density,
    # velocity, temperature, stress and heat flux (quadrature of eq. (3)-(4))
    al = orc.alpha_list(M)
    fields = [1.3, 0.12, -0.07, 0.9, 0.05, -0.03, 0.02, 0.04, -0.06]
    r = R.fields_to_record(M, al, fields)
    rho, u1, u2, th, s11, s12, s22, q1, q2 = fields
    g = HQ.Grid(r[:2], r[2])
    fv = HQ.function_values(al, r[3:], r[:2], r[2], g.xi)
    c = g.xi - np.array([u1, u2, 0.0])
    assert abs(np.sum(g.W * fv) - rho) < 1e-13
    assert np.allclose([np.sum(g.W * fv * g.xi[:, d]) / rho for d in range(3)], [u1, u2, 0.0],
                       atol=1e-13)
    assert abs(np.sum(g.W * fv * (c ** 2).sum(axis=1)) / (3 * rho) - th) < 1e-13
    sig = lambda i, j: np.sum(g.W * fv * c[:, i] * c[:, j]) - rho * th * (i == j)
    assert np.allclose([sig(0, 0), sig(0, 1), sig(1, 1), sig(2, 2), sig(0, 2), sig(1, 2)],
                       [s11, s12, s22, -(s11 + s22), 0.0, 0.0], atol=1e-13)
    q = [0.5 * np.sum(g.W * fv * (c ** 2).sum(axis=1) * c[:, i]) for i in range(3)]
    assert np.allclose(q, [q1, q2, 0.0], atol=1e-13)
    # and the oracle's own macroscopic map agrees
    mac = orc.macro(M, r)
    assert np.allclose(mac[[0, 1, 2, 3, 4, 5, 6, 8, 9]], fields, atol=1e-14)
