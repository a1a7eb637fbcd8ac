"""Seeded synthetic inputs: workload specifications and cell states.

This module holds no arithmetic of the method.  It names the cavity workloads
(dimensionless analogues of the paper's single lid-driven, Sec. 4.1, and
bottom-heated, Sec. 4.3, cavities) and draws seeded states that satisfy the
constraints a state of the Grad-basis expansion must satisfy (Sec. 2.2,
eq. (10)): f_0 = rho > 0, f_{e_i} = 0, f_{2e_1} + f_{2e_2} + f_{2e_3} = 0,
theta > 0, and every coefficient with odd alpha_3 equal to zero (the flow is
two-dimensional and even in xi_3).

Record layout used here: ``[u1, u2, theta, f_0, ..., f_{N-1}]`` per cell,
coefficients in the graded order (|alpha| ascending; within one degree alpha_1
descending, then alpha_2 descending).
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Defaults shared by every workload (Sec. 4: CFL 0.9, s1 = s2 = 2, s3 = 4,
# omega = 0.81, beta = 1, V-cycles, argon Pr = 2/3 for Shakhov).
_BASE = dict(
    nx=32, ny=32, lx=1.0, ly=1.0, M=3, collision=0, Pr=1.0, Kn=0.1, omega=0.81, beta=1.0,
    order=1, limiter=0, cfl=0.9, nu_dt_cap=1.0,
    wall_u=[0.0, 0.0, 0.0, 0.0], wall_theta=[1.0, 1.0, 1.0, 1.0],
    levels=2, s1=2, s2=2, s3=4, gamma=1, mass0=1.0, precision=0,
)

# Walls are ordered S, E, N, W; wall_u is the tangential speed (x for S/N,
# y for E/W).
WORKLOADS = {
    # lid-driven cavity, plain FP64: 32x32, BGK, Kn 0.1, M = 3, 1st order,
    # lid (0.2, 0, 0), 2-level V-cycle, residual 1e-8
    "lid32_bgk_m3": dict(nx=32, ny=32, M=3, collision=0, Pr=1.0, Kn=0.1, order=1,
                         wall_u=[0.0, 0.0, 0.2, 0.0], levels=2, tol=1e-8),
    # lid-driven cavity: 128x128, Shakhov Pr 2/3, Kn 0.075, M = 5, 2nd order
    # minmod, lid (0.5, 0, 0), 4-level V-cycle, residual 1e-10
    "lid128_shakhov_m5": dict(nx=128, ny=128, M=5, collision=1, Pr=2.0 / 3.0, Kn=0.075, order=2,
                              limiter=0, wall_u=[0.0, 0.0, 0.5, 0.0], levels=4, tol=1e-10),
    # the same cavity with the paper's unlimited central slopes (eq. (15)):
    # with minmod the residual of this case stalls near 5e-6 (limiter
    # switching), so time-to-residual is measured on this variant
    "lid128_shakhov_m5_central": dict(nx=128, ny=128, M=5, collision=1, Pr=2.0 / 3.0, Kn=0.075,
                                      order=2, limiter=1, wall_u=[0.0, 0.0, 0.5, 0.0], levels=4,
                                      tol=1e-10),
    # bottom-heated cavity: 256x256, Shakhov, Kn 0.05 or 0.2, M = 8, 2nd
    # order with the paper's central slopes (eq. (15)), bottom wall theta 2,
    # others 1, static, 5-level V-cycle
    "heated256_shakhov_m8_kn005": dict(nx=256, ny=256, M=8, collision=1, Pr=2.0 / 3.0, Kn=0.05,
                                       order=2, limiter=1, wall_theta=[2.0, 1.0, 1.0, 1.0],
                                       levels=5, tol=1e-8),
    "heated256_shakhov_m8_kn02": dict(nx=256, ny=256, M=8, collision=1, Pr=2.0 / 3.0, Kn=0.2,
                                      order=2, limiter=1, wall_theta=[2.0, 1.0, 1.0, 1.0],
                                      levels=5, tol=1e-8),
    # the paper's Table-1 setup in dimensionless form: Shakhov, Kn 0.1, M = 5,
    # 1st order, U_W = 50 m/s at 273 K (0.2097 in sqrt(R T0) units), 8x8
    # coarsest grid
    "paper_table1_32": dict(nx=32, ny=32, M=5, collision=1, Pr=2.0 / 3.0, Kn=0.1, order=1,
                            wall_u=[0.0, 0.0, 0.2097, 0.0], levels=3, tol=1e-8),
    # the ES-BGK model (eq. (7)) on the same single lid (Table 4 setup):
    # Pr 2/3 and beta = Pr in the collision frequency (Sec. 4), 64x64, M = 5
    "esbgk64_m5_kn01": dict(nx=64, ny=64, M=5, collision=2, Pr=2.0 / 3.0, beta=2.0 / 3.0, Kn=0.1,
                            order=1, wall_u=[0.0, 0.0, 0.2097, 0.0], levels=4, tol=1e-8),
    # four-sided lid-driven cavity with anti-parallel wall motion (Sec. 4.2):
    # top moves right and the right wall up at U_W (50 m/s at 273 K, 0.2097),
    # bottom and left walls the opposite way; Shakhov, Kn 0.777, M = 5, 1st
    # order, 64x64 with an 8x8 coarsest grid, residual 1e-8
    "four_sided64_shakhov_m5": dict(nx=64, ny=64, M=5, collision=1, Pr=2.0 / 3.0, Kn=0.777,
                                    order=1, wall_u=[-0.2097, 0.2097, 0.2097, -0.2097], levels=4,
                                    tol=1e-8),
}


def spec(name: str | None = None, **overrides) -> dict:
    """Full problem specification: defaults, then a named workload, then overrides."""
    s = copy.deepcopy(_BASE)
    s["tol"] = 1e-8
    if name is not None:
        s.update(copy.deepcopy(WORKLOADS[name]))
    s.update(overrides)
    return s


def nalpha(M: int) -> int:
    return (M + 1) * (M + 2) * (M + 3) // 6


def alpha_list(M: int) -> np.ndarray:
    """The graded index order of the coefficient vector."""
    out = []
    for n in range(M + 1):
        for a1 in range(n, -1, -1):
            for a2 in range(n - a1, -1, -1):
                out.append((a1, a2, n - a1 - a2))
    return np.array(out, dtype=np.int32)


def level_shape(s: dict, level: int) -> tuple[int, int]:
    return s["nx"] >> level, s["ny"] >> level


def maxwellian_state(s: dict, level: int = 0, rho: float = 1.0, u=(0.0, 0.0), theta: float = 1.0):
    """Global Maxwellian: every cell (u, theta) and f_0 = rho, all else zero."""
    nx, ny = level_shape(s, level)
    st = np.zeros((ny, nx, nalpha(s["M"]) + 3))
    st[..., 0], st[..., 1], st[..., 2], st[..., 3] = u[0], u[1], theta, rho
    return st


def random_state(s: dict, level: int = 0, seed: int = 0, amp: float = 0.05, smooth: bool = True):
    """A seeded, physically admissible, non-equilibrium state.

    Smooth large-scale fields plus cell noise for (rho, u, theta); higher
    coefficients drawn with scale amp * rho * theta^(n/2) / 2^n for degree n,
    then the constraints of eq. (10) and xi_3-parity imposed.
    """
    rng = np.random.default_rng(seed)
    nx, ny = level_shape(s, level)
    M = s["M"]
    al = alpha_list(M)
    N = len(al)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)

    def field(base, scale):
        ph = rng.uniform(0, 2 * math.pi, size=4)
        v = base + scale * (0.6 * np.sin(2 * math.pi * X + ph[0]) * np.cos(math.pi * Y + ph[1])
                            + 0.4 * np.sin(3 * math.pi * Y + ph[2]) * np.cos(2 * math.pi * X + ph[3]))
        if not smooth:
            v = base + scale * rng.uniform(-1, 1, size=(ny, nx))
        return v + 0.1 * scale * rng.uniform(-1, 1, size=(ny, nx))

    rho = field(1.0, 4 * amp)
    th = field(1.0, 4 * amp)
    st = np.zeros((ny, nx, N + 3))
    st[..., 0] = field(0.0, 2 * amp)
    st[..., 1] = field(0.0, 2 * amp)
    st[..., 2] = th
    st[..., 3] = rho
    for k in range(1, N):
        n = int(al[k].sum())
        st[..., 3 + k] = field(0.0, amp * 2.0 ** (-n)) * rho * th ** (n / 2)
    for k in range(N):
        a1, a2, a3 = (int(v) for v in al[k])
        if a3 % 2 == 1 or a1 + a2 + a3 == 1:
            st[..., 3 + k] = 0.0
    i200 = [k for k in range(N) if tuple(al[k]) == (2, 0, 0)][0]
    i020 = [k for k in range(N) if tuple(al[k]) == (0, 2, 0)][0]
    i002 = [k for k in range(N) if tuple(al[k]) == (0, 0, 2)][0]
    st[..., 3 + i002] = -(st[..., 3 + i200] + st[..., 3 + i020])
    return st


def random_rhs(s: dict, level: int, seed: int, amp: float = 0.02):
    """A seeded right-hand-side record set (basis + coefficients) for coarse-level tests."""
    st = random_state(s, level, seed=seed, amp=amp)
    rng = np.random.default_rng(seed + 7919)
    N = st.shape[-1] - 3
    al = alpha_list(s["M"])
    coef = amp * rng.standard_normal(st[..., 3:].shape)
    odd = al[:, 2] % 2 == 1
    coef[..., odd] = 0.0
    st[..., 3:] = coef[..., :N]
    return st


# ---------------------------------------------------------------------------
# Cavity parameter draws and the warm-start network's inputs
# ---------------------------------------------------------------------------

# Layer widths of the warm-start network: 8 inputs, three hidden layers of
# 256, 9 outputs (rho, u1, u2, theta, sigma11, sigma12, sigma22, q1, q2).
MLP_LAYERS = (8, 256, 256, 256, 9)
FIELD_NAMES = ("rho", "u1", "u2", "theta", "s11", "s12", "s22", "q1", "q2")
FEATURE_NAMES = ("log10Kn", "lid", "thS", "thE", "thN", "thW", "x", "y")

# seeds of the draws: training set, held-out set, network initialisation
SEED_TRAIN, SEED_TEST, SEED_INIT = 220613165, 220613166, 220613167
SEED_BATCH = 220613164


def levels_for_side(side: int, coarsest: int = 8) -> int:
    """Multigrid levels of a square grid: coarsen while the side is even and
    half of it is at least `coarsest` (64 -> 4, 96 -> 4, 128 -> 5, 192 -> 5,
    256 -> 6)."""
    k = 1
    while side % 2 == 0 and side // 2 >= coarsest:
        side //= 2
        k += 1
    return k


def cavity_draws(n: int, seed: int, sides=(64, 96, 128, 192, 256), Ms=(3, 5, 8), levels=None,
                 kn_range=(0.01, 1.0), lid_range=(0.1, 0.5), **overrides) -> list[dict]:
    """Lid-driven cavities with randomly drawn parameters, in the draw order
    (side, Kn, lid speed, M, collision model) per cavity: side uniform over
    `sides`, Kn log-uniform, lid speed uniform, M uniform over `Ms`, BGK or
    Shakhov (Pr 2/3) with probability 1/2; second order (central slopes),
    walls at theta = 1; levels from the side (levels_for_side) unless given."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        side = int(rng.choice(sides))
        kn = float(np.exp(rng.uniform(np.log(kn_range[0]), np.log(kn_range[1]))))
        lid = float(rng.uniform(*lid_range))
        M = int(rng.choice(Ms))
        coll = int(rng.integers(0, 2))
        d = dict(nx=side, ny=side, M=M, collision=coll, Pr=2.0 / 3.0 if coll else 1.0, Kn=kn,
                 order=2, limiter=1, wall_u=[0.0, 0.0, lid, 0.0],
                 levels=levels if levels else levels_for_side(side), tol=1e-8)
        d.update(overrides)
        out.append(spec(None, **d))
    return out


def mlp_features(s: dict, nx: int, ny: int) -> np.ndarray:
    """Network inputs of every cell centre of an nx x ny grid over the
    cavity of spec s: (log10 Kn, lid speed, wall theta S/E/N/W, x, y), rows in
    row-major cell order, float32."""
    x = (np.arange(nx) + 0.5) / nx * s["lx"]
    y = (np.arange(ny) + 0.5) / ny * s["ly"]
    X, Y = np.meshgrid(x, y)
    F = np.zeros((ny * nx, 8), dtype=np.float32)
    F[:, 0] = math.log10(s["Kn"])
    F[:, 1] = s["wall_u"][2]
    F[:, 2:6] = np.asarray(s["wall_theta"], dtype=np.float32)
    F[:, 6] = X.ravel()
    F[:, 7] = Y.ravel()
    return F


def mlp_init(seed: int = SEED_INIT, layers=MLP_LAYERS) -> list[tuple[np.ndarray, np.ndarray]]:
    """Seeded initial parameters: per layer W (out x in) and b (out), uniform
    in +-1/sqrt(fan_in), float64."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(len(layers) - 1):
        a = 1.0 / math.sqrt(layers[k])
        W = rng.uniform(-a, a, size=(layers[k + 1], layers[k]))
        b = rng.uniform(-a, a, size=layers[k + 1])
        out.append((W, b))
    return out
