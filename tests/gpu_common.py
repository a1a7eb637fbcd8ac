"""Helpers shared by the GPU tests: contexts, layout conversion, error metrics."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2206_13164_amd import inputs as I

# Tolerances (FP64): one application of an operator, sweep, restriction or
# correction from identical inputs agrees to 1e-12; fields after the same
# number of V-cycles agree to 1e-10 (the parity bounds of this library).
TOL_STEP = 1e-12
TOL_CONVERGED = 1e-10


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_13164_amd import nrxx as N
    N.load()  # a missing library is an error, not a skip
    return torch


def context(spec):
    from paper_2206_13164_amd import nrxx as N
    return N.Context(spec)


def state_err(a, b, M):
    """max over cells of |du|/sqrt(th), |dth|/th, |df_alpha|/(rho th^{|alpha|/2})."""
    n = I.alpha_list(M).sum(axis=1)
    rho, th = b[..., 3], b[..., 2]
    eu = (np.abs(a[..., :2] - b[..., :2]).max(axis=-1) / np.sqrt(th)).max()
    et = (np.abs(a[..., 2] - b[..., 2]) / th).max()
    scale = rho[..., None] * th[..., None] ** (n / 2.0)
    ef = (np.abs(a[..., 3:] - b[..., 3:]) / scale).max()
    return float(max(eu, et, ef))


def record_err(a, b, floor=1e-3):
    """Residual-type records: basis parameters must agree; coefficients are
    compared cell by cell, each difference divided by the largest coefficient
    of that cell's reference record (bounded below by `floor` times the
    largest of the whole level, so that a cell whose residual vanishes is
    compared at the level's scale rather than at zero)."""
    eb = np.abs(a[..., :3] - b[..., :3]).max()
    cell = np.abs(b[..., 3:]).max(axis=-1, keepdims=True)
    scale = np.maximum(cell, max(floor * float(cell.max()), 1e-300))
    ec = (np.abs(a[..., 3:] - b[..., 3:]) / scale).max()
    return float(max(eb, ec))
