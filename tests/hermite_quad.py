"""Independent evaluation of Hermite expansions by quadrature (test helper).

Written from the definitions of Sec. 2.2 only (basis function H_alpha^[u,th],
coefficients by orthogonality), with numpy's probabilists' Hermite routines;
it shares nothing with the oracle's recurrences.  Used to pin the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import hermite_e as He

NQ = 24  # Gauss-HermiteE nodes per dimension (exact for degree <= 47)


def _he(n, x):
    c = np.zeros(n + 1)
    c[n] = 1.0
    return He.hermeval(x, c)


class Grid:
    """Tensor Gauss-HermiteE grid adapted to the basis [u, th]:
    xi = u + sqrt(th) v, with sum(W * g(xi)) = int g(xi) dxi for g polynomial
    times the Maxwellian weight of [u, th]."""

    def __init__(self, u, th, nq=NQ):
        v, w = He.hermegauss(nq)
        w = w / math.sqrt(2 * math.pi)
        self.u = np.array([u[0], u[1], 0.0])
        self.th = th
        V = np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=-1).reshape(-1, 3)
        W = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
        self.v = V                      # nodes in the scaled variable
        self.xi = self.u + math.sqrt(th) * V
        # int g(xi) dxi = th^{3/2} int g(u + sqrt(th) v) dv; the Gauss weight
        # already accounts for e^{-|v|^2/2} / (2 pi)^{3/2}
        self.W = W * (2 * math.pi) ** 1.5 * th ** 1.5 * np.exp(0.5 * (V ** 2).sum(axis=1))


def basis_values(alpha, u, th, xi):
    """H_alpha^[u,th](xi) for each row of xi (m = 1)."""
    uu = np.array([u[0], u[1], 0.0])
    v = (xi - uu) / np.sqrt(th)
    out = np.exp(-0.5 * (v ** 2).sum(axis=1)) / (2 * math.pi * th) ** 1.5
    out = out * th ** (-sum(alpha) / 2.0)
    for d in range(3):
        out = out * _he(int(alpha[d]), v[:, d])
    return out


def function_values(alist, f, u, th, xi):
    """f(xi) = sum_alpha f_alpha H_alpha^[u,th](xi)."""
    out = np.zeros(xi.shape[0], dtype=np.result_type(f, xi, float))
    for k, a in enumerate(alist):
        if f[k] != 0:
            out = out + f[k] * basis_values(a, u, th, xi)
    return out


def project(alist, g_values, grid: Grid, u, th):
    """Coefficients of g in F_M^[u,th]: f_alpha = th^{|alpha|/2}/alpha! int He_alpha(v) g dxi.
    `grid` supplies nodes/weights; g must be given at grid.xi."""
    uu = np.array([u[0], u[1], 0.0])
    v = (grid.xi - uu) / math.sqrt(th)
    out = np.zeros(len(alist), dtype=g_values.dtype)
    for k, a in enumerate(alist):
        h = np.ones(v.shape[0])
        for d in range(3):
            h = h * _he(int(a[d]), v[:, d])
        fac = math.factorial(a[0]) * math.factorial(a[1]) * math.factorial(a[2])
        out[k] = th ** (sum(a) / 2.0) / fac * np.sum(grid.W * h * g_values)
    return out


def moments(alist, f, u, th):
    """rho, rho u (3), int |xi|^2 f, by quadrature."""
    g = Grid(u, th)
    fv = function_values(alist, f, u, th, g.xi)
    rho = np.sum(g.W * fv)
    mom = np.array([np.sum(g.W * fv * g.xi[:, d]) for d in range(3)])
    en = np.sum(g.W * fv * (g.xi ** 2).sum(axis=1))
    return rho, mom, en
