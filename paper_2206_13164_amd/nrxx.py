"""Python binding of ``libnrxx.so`` (the C ABI of ``include/nrxx.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory and the stream.  Importing works without a
GPU; creating a context needs the built library and a GPU, and fails loudly
otherwise (there is no fallback).

Device state tensors have shape ``(ny, nx, record_stride(M))`` and dtype
float64; record layout ``[u1, u2, theta, f_0 .. f_{N-1}, padding]``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnrxx.so")

NRXX_OK, NRXX_EINVAL, NRXX_ENONPHYS, NRXX_EDIVERGED = 0, -1, -2, -3
NRXX_ENOMEM, NRXX_EHIP, NRXX_EMAXIT = -4, -5, -6
STATUS = {0: "NRXX_OK", -1: "NRXX_EINVAL", -2: "NRXX_ENONPHYS", -3: "NRXX_EDIVERGED",
          -4: "NRXX_ENOMEM", -5: "NRXX_EHIP", -6: "NRXX_EMAXIT"}

c_int, c_double, c_void_p = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p


class Problem(ctypes.Structure):
    _fields_ = [
        ("nx", c_int), ("ny", c_int), ("lx", c_double), ("ly", c_double),
        ("M", c_int), ("collision", c_int),
        ("Pr", c_double), ("Kn", c_double), ("omega", c_double), ("beta", c_double),
        ("order", c_int), ("limiter", c_int), ("cfl", c_double), ("nu_dt_cap", c_double),
        ("wall_u", c_double * 4), ("wall_theta", c_double * 4),
        ("levels", c_int), ("s1", c_int), ("s2", c_int), ("s3", c_int), ("gamma", c_int),
        ("mass0", c_double), ("precision", c_int), ("schedule", c_int),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [("M", c_int), ("order", c_int), ("problems", c_int), ("team_width", c_int),
                ("grid", c_int), ("unit_order", c_int), ("split", c_int), ("block_ms", c_double),
                ("kernel", c_int), ("rows_per_sync", c_int)]


_PP = ctypes.POINTER(c_void_p)

EXPORTS = {
    "nrxx_record_stride": (c_int, [c_int]),
    "nrxx_create": (c_int, [ctypes.POINTER(Problem), c_void_p, ctypes.POINTER(c_void_p)]),
    "nrxx_destroy": (c_int, [c_void_p]),
    "nrxx_last_error": (ctypes.c_char_p, [c_void_p]),
    "nrxx_level_shape": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "nrxx_level_schedule": (c_int, [c_void_p, c_int]),
    "nrxx_init_maxwellian": (c_int, [c_void_p, c_int, c_void_p, c_double, c_double, c_double, c_double]),
    "nrxx_residual": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "nrxx_residual_noalloc": (c_int, [ctypes.POINTER(Problem), c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p, ctypes.POINTER(c_double), c_void_p]),
    "nrxx_sweep": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int]),
    "nrxx_restrict": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nrxx_fas_rhs": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "nrxx_correct": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "nrxx_euler": (c_int, [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(c_double)]),
    "nrxx_mass": (c_int, [c_void_p, c_int, c_void_p, ctypes.POINTER(c_double)]),
    "nrxx_fas_vcycle": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "nrxx_solve": (c_int, [c_void_p, c_void_p, c_double, c_int, c_double, ctypes.POINTER(c_int),
                           c_void_p]),
    "nrxx_sweep_stats": (c_int, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                 ctypes.POINTER(c_double), c_int]),
    "nrxx_batch_create": (c_int, [ctypes.POINTER(Problem), c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "nrxx_batch_destroy": (c_int, [c_void_p]),
    "nrxx_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "nrxx_batch_groups": (c_int, [c_void_p]),
    "nrxx_batch_get_tuning": (c_int, [c_void_p, c_int, ctypes.POINTER(BatchTuning)]),
    "nrxx_batch_set_tuning": (c_int, [c_void_p, c_int, ctypes.POINTER(BatchTuning)]),
    "nrxx_batch_autotune": (c_int, [c_void_p, _PP]),
    "nrxx_batch_init_maxwellian": (c_int, [c_void_p, _PP, c_double, c_double, c_double, c_double]),
    "nrxx_batch_residual_norms": (c_int, [c_void_p, _PP, c_void_p]),
    "nrxx_batch_sweep": (c_int, [c_void_p, _PP, c_int]),
    "nrxx_batch_vcycle": (c_int, [c_void_p, _PP, c_void_p]),
    "nrxx_batch_solve": (c_int, [c_void_p, _PP, c_double, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "nrxx_batch_stats": (c_int, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double), c_int]),
    "nrxx_batch_set_timing": (c_int, [c_void_p, c_int]),
    "nrxx_batch_kernel_stats": (c_int, [c_void_p, c_int, ctypes.POINTER(c_double),
                                        ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                        ctypes.POINTER(c_double), c_int]),
    "nrxx_set_wait_limit": (c_int, [c_void_p, c_double]),
    "nrxx_batch_set_wait_limit": (c_int, [c_void_p, c_double]),
    "nrxx_init_fields": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    "nrxx_state_fields": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "nrxx_mlp_create": (c_int, [c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "nrxx_mlp_destroy": (c_int, [c_void_p]),
    "nrxx_mlp_last_error": (ctypes.c_char_p, [c_void_p]),
    "nrxx_mlp_param_count": (ctypes.c_int64, [c_void_p]),
    "nrxx_mlp_set_params": (c_int, [c_void_p, c_void_p]),
    "nrxx_mlp_get_params": (c_int, [c_void_p, c_void_p]),
    "nrxx_mlp_set_scaling": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nrxx_mlp_forward": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "nrxx_mlp_gradients": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                   ctypes.POINTER(c_double)]),
    "nrxx_mlp_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float,
                                    ctypes.POINTER(c_double)]),
}

_lib = None


def load():
    """Load libnrxx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2206_13164_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class NrxxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def record_stride(M: int) -> int:
    return load().nrxx_record_stride(M)


def problem(spec) -> Problem:
    p = Problem()
    for name, _ in Problem._fields_:
        if name == "schedule":
            p.schedule = int(spec.get("schedule", 0))
            continue
        v = spec[name]
        if name in ("wall_u", "wall_theta"):
            getattr(p, name)[:] = [float(x) for x in v]
        else:
            setattr(p, name, v)
    return p


def _ptr(t):
    if t is None:
        return None
    return c_void_p(t.data_ptr())


NOALLOC_MAX_CELLS = 262144  # NRXX_NOALLOC_MAX_CELLS of include/nrxx.h


def residual_noalloc(spec, state, level=0, rhs=None, out=None, norm_dev=None, host_norm=True,
                     stream=None):
    """nrxx_residual_noalloc: the defect (into `out`, may be None) and the
    eq. (28) norm of `state` on `level` of the problem `spec`, without a
    context and without allocating.  `norm_dev` (a 1-element float64 CUDA
    tensor, may be None) receives the norm on the device; with host_norm the
    call synchronises and returns it (else returns None)."""
    import torch
    L = load()
    P = problem(spec)
    if stream is None:
        stream = torch.cuda.current_stream()
    nrm = c_double()
    rc = L.nrxx_residual_noalloc(ctypes.byref(P), level, _ptr(state), _ptr(rhs), _ptr(out),
                                 _ptr(norm_dev), ctypes.byref(nrm) if host_norm else None,
                                 c_void_p(stream.cuda_stream))
    if rc != NRXX_OK:
        raise NrxxError(rc, L.nrxx_last_error(None).decode())
    return nrm.value if host_norm else None


class Context:
    """Owns an nrxx_ctx.  Tensors passed in must be float64 CUDA tensors laid
    out as (ny, nx, record_stride(M)) for the level they belong to."""

    def __init__(self, spec, stream=None):
        import torch
        self.torch = torch
        L = load()
        self.spec = dict(spec)
        self.M = int(spec["M"])
        self.stride = record_stride(self.M)
        self.P = problem(spec)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        rc = L.nrxx_create(ctypes.byref(self.P), c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != NRXX_OK:
            raise NrxxError(rc, L.nrxx_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().nrxx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, allow=()):
        if rc != NRXX_OK and rc not in allow:
            raise NrxxError(rc, load().nrxx_last_error(self.h).decode())
        return rc

    # -- helpers -----------------------------------------------------------
    def level_shape(self, level):
        nx, ny = c_int(), c_int()
        self._chk(load().nrxx_level_shape(self.h, level, ctypes.byref(nx), ctypes.byref(ny)))
        return nx.value, ny.value

    def level_schedule(self, level):
        rc = load().nrxx_level_schedule(self.h, level)
        self._chk(rc if rc < 0 else 0)
        return rc

    def empty(self, level=0):
        nx, ny = self.level_shape(level)
        return self.torch.zeros((ny, nx, self.stride), dtype=self.torch.float64, device="cuda")

    def to_device(self, rec: np.ndarray):
        """(ny, nx, N+3) host records -> padded device tensor."""
        ny, nx, r = rec.shape
        t = self.torch.zeros((ny, nx, self.stride), dtype=self.torch.float64)
        t[..., :r] = self.torch.from_numpy(np.ascontiguousarray(rec))
        return t.to("cuda")

    @staticmethod
    def to_host(t, nrec: int) -> np.ndarray:
        return t[..., :nrec].detach().cpu().numpy().copy()

    # -- C ABI -------------------------------------------------------------
    def init_maxwellian(self, state, level=0, rho=1.0, u=(0.0, 0.0), theta=1.0):
        self._chk(load().nrxx_init_maxwellian(self.h, level, _ptr(state), rho, u[0], u[1], theta))

    def residual(self, state, level=0, rhs=None, out=None, want_norm=True):
        nrm = c_double()
        self._chk(load().nrxx_residual(self.h, level, _ptr(state), _ptr(rhs), _ptr(out),
                                       ctypes.byref(nrm) if want_norm else None))
        return nrm.value if want_norm else None

    def sweep(self, state, level=0, rhs=None, dir_mask=15, nsteps=1):
        self._chk(load().nrxx_sweep(self.h, level, _ptr(state), _ptr(rhs), dir_mask, nsteps))

    def restrict(self, fine, level_fine=0, fineR=None, coarse=None, coarseR=None):
        self._chk(load().nrxx_restrict(self.h, level_fine, _ptr(fine), _ptr(fineR), _ptr(coarse),
                                       _ptr(coarseR)))

    def fas_rhs(self, coarse, coarseR, rhs, level_coarse):
        self._chk(load().nrxx_fas_rhs(self.h, level_coarse, _ptr(coarse), _ptr(coarseR), _ptr(rhs)))

    def correct(self, fine, coarse_new, coarse_old, level_fine=0):
        self._chk(load().nrxx_correct(self.h, level_fine, _ptr(fine), _ptr(coarse_new), _ptr(coarse_old)))

    def mass(self, state, level=0):
        m = c_double()
        self._chk(load().nrxx_mass(self.h, level, _ptr(state), ctypes.byref(m)))
        return m.value

    def euler(self, state, nsteps=1, level=0):
        """`nsteps` forward Euler steps with the global time step (the
        explicit time-marching baseline); returns the last step's dt."""
        dt = c_double()
        self._chk(load().nrxx_euler(self.h, level, _ptr(state), nsteps, ctypes.byref(dt)))
        return dt.value

    def fas_vcycle(self, state, want_norm=True):
        nrm = c_double()
        self._chk(load().nrxx_fas_vcycle(self.h, _ptr(state), ctypes.byref(nrm) if want_norm else None))
        return nrm.value if want_norm else None

    def solve(self, state, tol, max_cycles, ref_norm=0.0):
        cyc = c_int()
        hist = np.zeros(max_cycles + 1)
        rc = load().nrxx_solve(self.h, _ptr(state), tol, max_cycles, ref_norm, ctypes.byref(cyc),
                               hist.ctypes.data_as(c_void_p))
        self._chk(rc, allow=(NRXX_EMAXIT,))
        return rc, cyc.value, hist[: cyc.value + 1]

    def init_fields(self, state, fields):
        """fields: float32 CUDA tensor (fny, fnx, 9) on a grid dividing the finest."""
        fny, fnx, _ = fields.shape
        self._chk(load().nrxx_init_fields(self.h, _ptr(state), _ptr(fields), fnx, fny))

    def state_fields(self, state, level=0):
        nx, ny = self.level_shape(level)
        out = self.torch.zeros((ny, nx, 9), dtype=self.torch.float32, device="cuda")
        self._chk(load().nrxx_state_fields(self.h, level, _ptr(state), _ptr(out)))
        return out

    def set_wait_limit(self, seconds):
        self._chk(load().nrxx_set_wait_limit(self.h, float(seconds)))

    def sweep_stats(self, reset=False):
        """(device ms in sweep kernels, cell updates, sweep kernel launches)."""
        ms, cells, launches = c_double(), c_double(), c_double()
        self._chk(load().nrxx_sweep_stats(self.h, ctypes.byref(ms), ctypes.byref(cells),
                                          ctypes.byref(launches), int(reset)))
        return ms.value, cells.value, launches.value


class Batch:
    """Owns an nrxx_batch: many problems (specs) solved together.  States are
    lists of float64 CUDA tensors, one per problem, shaped
    (ny, nx, record_stride(M)) for that problem's finest level."""

    def __init__(self, specs, stream=None):
        import torch
        self.torch = torch
        L = load()
        self.specs = [dict(x) for x in specs]
        self.n = len(self.specs)
        arr = (Problem * self.n)(*[problem(x) for x in self.specs])
        self._arr = arr
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        rc = L.nrxx_batch_create(arr, self.n, c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != NRXX_OK:
            raise NrxxError(rc, L.nrxx_batch_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().nrxx_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, allow=()):
        if rc != NRXX_OK and rc not in allow:
            raise NrxxError(rc, load().nrxx_batch_last_error(self.h).decode())
        return rc

    def _ptrs(self, states):
        if len(states) != self.n:
            raise ValueError("need one state per problem")
        return (c_void_p * self.n)(*[t.data_ptr() for t in states])

    def empty_states(self):
        out = []
        for x in self.specs:
            st = record_stride(int(x["M"]))
            out.append(self.torch.zeros((x["ny"], x["nx"], st), dtype=self.torch.float64,
                                        device="cuda"))
        return out

    def groups(self):
        return load().nrxx_batch_groups(self.h)

    def tuning(self, group):
        t = BatchTuning()
        self._chk(load().nrxx_batch_get_tuning(self.h, group, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in BatchTuning._fields_}

    def set_tuning(self, group, team_width, grid, unit_order, split=1, kernel=0, rows_per_sync=1):
        t = BatchTuning()
        t.team_width, t.grid, t.unit_order, t.split = team_width, grid, unit_order, split
        t.kernel, t.rows_per_sync = kernel, rows_per_sync
        self._chk(load().nrxx_batch_set_tuning(self.h, group, ctypes.byref(t)))

    def autotune(self, states):
        self._chk(load().nrxx_batch_autotune(self.h, self._ptrs(states)))

    def init_maxwellian(self, states, rho=1.0, u=(0.0, 0.0), theta=1.0):
        self._chk(load().nrxx_batch_init_maxwellian(self.h, self._ptrs(states), rho, u[0], u[1], theta))

    def residual_norms(self, states):
        out = np.zeros(self.n)
        self._chk(load().nrxx_batch_residual_norms(self.h, self._ptrs(states),
                                                   out.ctypes.data_as(c_void_p)))
        return out

    def sweep(self, states, nsteps=1):
        self._chk(load().nrxx_batch_sweep(self.h, self._ptrs(states), nsteps))

    def vcycle(self, states):
        out = np.zeros(self.n)
        self._chk(load().nrxx_batch_vcycle(self.h, self._ptrs(states), out.ctypes.data_as(c_void_p)))
        return out

    def solve(self, states, tol, max_cycles, use_graph=True):
        cyc = np.zeros(self.n, dtype=np.int32)
        nrm, ref = np.zeros(self.n), np.zeros(self.n)
        rc = load().nrxx_batch_solve(self.h, self._ptrs(states), tol, max_cycles, int(use_graph),
                                     cyc.ctypes.data_as(c_void_p), nrm.ctypes.data_as(c_void_p),
                                     ref.ctypes.data_as(c_void_p))
        self._chk(rc, allow=(NRXX_EMAXIT,))
        return rc, cyc, nrm, ref

    def set_wait_limit(self, seconds):
        self._chk(load().nrxx_batch_set_wait_limit(self.h, float(seconds)))

    def set_timing(self, on=True):
        self._chk(load().nrxx_batch_set_timing(self.h, int(bool(on))))

    def kernel_stats(self, group, reset=False):
        """(ms, launches, fine cell updates, coarse cell updates) of the
        group's sweep launches while timing is on."""
        v = [c_double() for _ in range(4)]
        self._chk(load().nrxx_batch_kernel_stats(self.h, group, *[ctypes.byref(x) for x in v],
                                                 int(reset)))
        return tuple(x.value for x in v)

    def stats(self, reset=False):
        ms, cells = c_double(), c_double()
        self._chk(load().nrxx_batch_stats(self.h, ctypes.byref(ms), ctypes.byref(cells), int(reset)))
        return ms.value, cells.value


class Mlp:
    """Owns an nrxx_mlp (the warm-start network).  Parameters travel as one
    flat float32 host array (per layer: W row-major, then b)."""

    def __init__(self, widths, max_rows, stream=None):
        import torch
        self.torch = torch
        L = load()
        self.widths = [int(w) for w in widths]
        w = (c_int * len(self.widths))(*self.widths)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        rc = L.nrxx_mlp_create(w, len(self.widths) - 1, int(max_rows), c_void_p(stream.cuda_stream),
                               ctypes.byref(h))
        if rc != NRXX_OK:
            raise NrxxError(rc, L.nrxx_mlp_last_error(None).decode())
        self.h = h
        self.n_params = int(L.nrxx_mlp_param_count(h))

    def close(self):
        if getattr(self, "h", None):
            load().nrxx_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != NRXX_OK:
            raise NrxxError(rc, load().nrxx_mlp_last_error(self.h).decode())

    @staticmethod
    def flatten(params):
        return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                               np.asarray(b, np.float32).ravel()])
                               for W, b in params]).astype(np.float32)

    def unflatten(self, flat):
        out, off = [], 0
        for k in range(len(self.widths) - 1):
            o, i = self.widths[k + 1], self.widths[k]
            W = flat[off:off + o * i].reshape(o, i)
            off += o * i
            out.append((W, flat[off:off + o]))
            off += o
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(self.flatten(params) if isinstance(params, list) else params,
                                    dtype=np.float32)
        assert flat.size == self.n_params
        self._chk(load().nrxx_mlp_set_params(self.h, flat.ctypes.data_as(c_void_p)))

    def get_params(self):
        flat = np.zeros(self.n_params, dtype=np.float32)
        self._chk(load().nrxx_mlp_get_params(self.h, flat.ctypes.data_as(c_void_p)))
        return flat

    def set_scaling(self, in_mean, in_std, out_mean, out_std):
        a = [np.ascontiguousarray(x, dtype=np.float32) for x in (in_mean, in_std, out_mean, out_std)]
        self._a = a
        self._chk(load().nrxx_mlp_set_scaling(self.h, *[x.ctypes.data_as(c_void_p) for x in a]))

    def forward(self, X):
        rows = X.shape[0]
        Y = self.torch.empty((rows, self.widths[-1]), dtype=self.torch.float32, device="cuda")
        self._chk(load().nrxx_mlp_forward(self.h, _ptr(X), rows, _ptr(Y)))
        return Y

    def gradients(self, X, T):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = c_double()
        self._chk(load().nrxx_mlp_gradients(self.h, _ptr(X), _ptr(T), X.shape[0],
                                            g.ctypes.data_as(c_void_p), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, X, T, lr, want_loss=False):
        loss = c_double()
        self._chk(load().nrxx_mlp_train_step(self.h, _ptr(X), _ptr(T), X.shape[0], float(lr),
                                             ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
