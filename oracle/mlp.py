"""FP64 CPU reference of the warm-start network and of the map from
macroscopic fields to a cell record.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the GPU
library).  Plain numpy in float64, written from the definitions:

* the network is a stack of affine layers z = a W^T + b, with the SiLU
  activation s(z) = z / (1 + exp(-z)) after every layer but the last;
* the loss is the mean of the squared differences over all rows and outputs;
* gradients are the chain rule written out layer by layer;
* the optimiser is Adam with bias correction (Kingma & Ba, 2015);
* fields -> record: the Grad-type closure that keeps rho, u, theta, the
  stress and the heat flux and sets every other coefficient to zero, in the
  basis [u, theta] (Sec. 2.2, eq. (10) and the moment relations of the paper).
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X):
    """params: list of (W [out x in], b [out]); X: rows x in.  Returns the
    output and the per-layer (input, pre-activation) pairs."""
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for k, (W, b) in enumerate(params):
        z = a @ W.T + b
        cache.append((a, z))
        a = z if k == len(params) - 1 else silu(z)
    return a, cache


def loss(Y, T):
    d = np.asarray(Y, dtype=np.float64) - T
    return float(np.mean(d * d))


def backward(params, cache, Y, T):
    """Gradients of loss(forward(X), T) with respect to every W and b."""
    Y = np.asarray(Y, dtype=np.float64)
    g = 2.0 * (Y - T) / Y.size  # d loss / d output
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        a, z = cache[k]
        W, _ = params[k]
        if k < len(params) - 1:
            g = g * silu_grad(z)
        grads[k] = (g.T @ a, g.sum(axis=0))
        g = g @ W
    return grads


def adam(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first); returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for p, gp, mp, vp in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mp = b1 * mp + (1.0 - b1) * gp
            vp = b2 * vp + (1.0 - b2) * gp * gp
            mh = mp / (1.0 - b1 ** t)
            vh = vp / (1.0 - b2 ** t)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), mp, vp))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def fields_to_record(M, alphas, fields):
    """Record [u1, u2, theta, f_alpha...] of a cell from its fields
    (rho, u1, u2, theta, sigma11, sigma12, sigma22, q1, q2): the basis is
    [u, theta]; f_0 = rho; f_{e_i} = 0; f_{e_i+e_j} = sigma_ij / (1 + delta_ij)
    with sigma33 = -(sigma11 + sigma22) (traceless stress); f_{3e_i} =
    f_{e_i+2e_d} (d != i) = q_i / 5, which gives back q_i =
    2 f_{3e_i} + sum_d f_{2e_d+e_i}; q3 = 0; everything else zero."""
    rho, u1, u2, th, s11, s12, s22, q1, q2 = [float(x) for x in fields]
    idx = {tuple(int(c) for c in a): k for k, a in enumerate(alphas)}
    f = np.zeros(len(alphas))
    f[idx[(0, 0, 0)]] = rho
    f[idx[(2, 0, 0)]] = s11 / 2.0
    f[idx[(0, 2, 0)]] = s22 / 2.0
    f[idx[(0, 0, 2)]] = -(s11 + s22) / 2.0
    f[idx[(1, 1, 0)]] = s12
    for i, q in ((0, q1), (1, q2)):
        for d in range(3):
            a = [0, 0, 0]
            a[i] += 1
            a[d] += 2
            f[idx[tuple(a)]] = q / 5.0
    return np.concatenate([[u1, u2, th], f])
