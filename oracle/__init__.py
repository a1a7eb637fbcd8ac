"""ctypes binding of the FP64 CPU oracle (``nrxx_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library never imports or
links it.  Records are numpy arrays of shape ``(ny, nx, N + 3)`` holding
``[u1, u2, theta, f_0 .. f_{N-1}]`` per cell, coefficients in the graded
order of ``alpha_list(M)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nrxx_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")

c_int, c_double = ctypes.c_int, ctypes.c_double
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class Problem(ctypes.Structure):
    _fields_ = [
        ("nx", c_int), ("ny", c_int), ("lx", c_double), ("ly", c_double),
        ("M", c_int), ("collision", c_int),
        ("Pr", c_double), ("Kn", c_double), ("omega", c_double), ("beta", c_double),
        ("order", c_int), ("limiter", c_int), ("cfl", c_double), ("nu_dt_cap", c_double),
        ("wall_u", c_double * 4), ("wall_theta", c_double * 4),
        ("levels", c_int), ("s1", c_int), ("s2", c_int), ("s3", c_int), ("gamma", c_int),
        ("mass0", c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Problem)
        sig = {
            "orc_nalpha": (c_int, [c_int]),
            "orc_alpha_list": (None, [c_int, np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")]),
            "orc_cmax": (c_double, [c_int]),
            "orc_basis_change": (None, [c_int, _dp, _dp, _dp, _dp]),
            "orc_xi_mult": (None, [c_int, c_int, _dp, _dp, _dp]),
            "orc_normalise": (c_int, [c_int, _dp]),
            "orc_macro": (None, [c_int, _dp, _dp]),
            "orc_collision": (None, [P, _dp, _dp]),
            "orc_regularisation": (None, [c_int, c_int, _dp, c_double, c_double, c_double, _dp]),
            "orc_wall_flux": (None, [P, c_int, _dp, _dp]),
            "orc_face_flux": (None, [P, c_int, _dp, _dp, _dp, _dp, _dp,
                                     ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
            "orc_cell_residual": (c_int, [P, c_int, _dp, c_int, c_int, _dp]),
            "orc_local_dt": (c_double, [P, c_int, _dp]),
            "orc_residual": (c_int, [P, c_int, _dp, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(c_double)]),
            "orc_norm": (c_double, [P, c_int, _dp]),
            "orc_mass": (c_double, [P, c_int, _dp]),
            "orc_sweep": (c_int, [P, c_int, _dp, ctypes.c_void_p, c_int, c_int, c_int]),
            "orc_restrict": (c_int, [P, c_int, _dp, ctypes.c_void_p, _dp, ctypes.c_void_p]),
            "orc_correct": (c_int, [P, c_int, _dp, _dp, _dp]),
            "orc_fas_rhs": (c_int, [P, c_int, _dp, _dp, _dp]),
            "orc_vcycle": (c_int, [P, c_int, _dp, ctypes.c_void_p]),
            "orc_mass_fix": (c_int, [P, _dp]),
            "orc_solve": (c_int, [P, _dp, c_double, c_int, c_double, ctypes.POINTER(c_int),
                                  ctypes.c_void_p]),
            "orc_euler_step": (c_int, [P, c_int, _dp, ctypes.POINTER(c_double)]),
            "orc_set_threads": (None, [c_int]),
            "orc_set_vcycle_wavefront": (None, [c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        _lib.orc_set_threads(1)
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def set_vcycle_wavefront(on: bool) -> None:
    """V-cycles sweep in anti-diagonal order (parallel over a diagonal's
    cells) instead of the serial order; the result is bitwise the same."""
    lib().orc_set_vcycle_wavefront(int(bool(on)))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def problem(spec) -> Problem:
    """Build the ctypes problem from a mapping with the fields of Problem."""
    p = Problem()
    for name, _ in Problem._fields_:
        v = spec[name]
        if name in ("wall_u", "wall_theta"):
            getattr(p, name)[:] = [float(x) for x in v]
        else:
            setattr(p, name, v)
    return p


def nalpha(M: int) -> int:
    return lib().orc_nalpha(M)


def alpha_list(M: int) -> np.ndarray:
    out = np.zeros((nalpha(M), 3), dtype=np.int32)
    lib().orc_alpha_list(M, out)
    return out


def cmax(n: int) -> float:
    return lib().orc_cmax(n)


def basis_change(M, f, frm, to):
    out = np.zeros(nalpha(M))
    lib().orc_basis_change(M, np.ascontiguousarray(f, dtype=np.float64),
                           np.asarray(frm, dtype=np.float64), np.asarray(to, dtype=np.float64), out)
    return out


def xi_mult(M, d, f, basis):
    out = np.zeros(nalpha(M))
    lib().orc_xi_mult(M, d, np.ascontiguousarray(f, dtype=np.float64),
                      np.asarray(basis, dtype=np.float64), out)
    return out


def normalise(M, rec):
    r = np.array(rec, dtype=np.float64)
    rc = lib().orc_normalise(M, r)
    return rc, r


def macro(M, rec):
    out = np.zeros(11)
    lib().orc_macro(M, np.ascontiguousarray(rec, dtype=np.float64), out)
    return out


def collision(P, rec):
    out = np.zeros(nalpha(P.M))
    lib().orc_collision(ctypes.byref(P), np.ascontiguousarray(rec, dtype=np.float64), out)
    return out


def regularisation(M, d, f, du1, du2, dth):
    out = np.zeros(nalpha(M))
    lib().orc_regularisation(M, d, np.ascontiguousarray(f, dtype=np.float64), du1, du2, dth, out)
    return out


def wall_flux(P, wall, rec):
    out = np.zeros(nalpha(P.M))
    lib().orc_wall_flux(ctypes.byref(P), wall, np.ascontiguousarray(rec, dtype=np.float64), out)
    return out


def face_flux(P, d, recL, recR, basis):
    N = nalpha(P.M)
    F, g = np.zeros(N), np.zeros(N)
    wm, wp = c_double(), c_double()
    lib().orc_face_flux(ctypes.byref(P), d, np.ascontiguousarray(recL, dtype=np.float64),
                        np.ascontiguousarray(recR, dtype=np.float64),
                        np.asarray(basis, dtype=np.float64), F, g, ctypes.byref(wm), ctypes.byref(wp))
    return F, g, wm.value, wp.value


def level_shape(P, level):
    return P.nx >> level, P.ny >> level


def cell_residual(P, level, st, i, j):
    out = np.zeros(nalpha(P.M))
    lib().orc_cell_residual(ctypes.byref(P), level, st, i, j, out)
    return out


def local_dt(P, level, rec):
    return lib().orc_local_dt(ctypes.byref(P), level, np.ascontiguousarray(rec, dtype=np.float64))


def residual(P, level, st, rhs=None):
    """Returns (r - R(f) records, norm)."""
    out = np.zeros_like(st)
    nrm = c_double()
    lib().orc_residual(ctypes.byref(P), level, st, _ptr(rhs), _ptr(out), ctypes.byref(nrm))
    return out, nrm.value


def norm(P, level, Rrec):
    return lib().orc_norm(ctypes.byref(P), level, np.ascontiguousarray(Rrec))


def mass(P, level, st):
    return lib().orc_mass(ctypes.byref(P), level, st)


def sweep(P, level, st, rhs=None, dir_mask=15, nsteps=1, wavefront=False):
    rc = lib().orc_sweep(ctypes.byref(P), level, st, _ptr(rhs), dir_mask, nsteps, int(wavefront))
    if rc:
        raise FloatingPointError("oracle sweep: non-physical state")
    return st


def restrict(P, level_fine, fine, fineR=None):
    nx, ny = level_shape(P, level_fine)
    R = fine.shape[-1]
    coarse = np.zeros((ny // 2, nx // 2, R))
    coarseR = np.zeros_like(coarse) if fineR is not None else None
    rc = lib().orc_restrict(ctypes.byref(P), level_fine, fine, _ptr(fineR), coarse, _ptr(coarseR))
    if rc:
        raise FloatingPointError("oracle restrict: non-physical state")
    return coarse, coarseR


def fas_rhs(P, level_coarse, coarse, coarseRbar):
    out = np.zeros_like(coarse)
    lib().orc_fas_rhs(ctypes.byref(P), level_coarse, coarse, coarseRbar, out)
    return out


def correct(P, level_fine, fine, coarse_new, coarse_old):
    return lib().orc_correct(ctypes.byref(P), level_fine, fine, coarse_new, coarse_old)


def vcycle(P, st, level=0, rhs=None):
    rc = lib().orc_vcycle(ctypes.byref(P), level, st, _ptr(rhs))
    if rc:
        raise FloatingPointError("oracle vcycle: non-physical state")
    return st


def mass_fix(P, st):
    return lib().orc_mass_fix(ctypes.byref(P), st)


def solve(P, st, tol, max_cycles, ref_norm=0.0):
    cyc = c_int()
    hist = np.zeros(max_cycles + 1)
    rc = lib().orc_solve(ctypes.byref(P), st, tol, max_cycles, ref_norm, ctypes.byref(cyc), _ptr(hist))
    return rc, cyc.value, hist[: cyc.value + 1]


def euler_step(P, st, level=0):
    dt = c_double()
    rc = lib().orc_euler_step(ctypes.byref(P), level, st, ctypes.byref(dt))
    if rc:
        raise FloatingPointError("oracle euler: non-physical state")
    return dt.value
