"""Error measures of the parity tests (no test of its own).

strict_err(a, b) is the largest of
  - the relative L2 error of every row of b (the last axis is the grid, the
    receiver or the component values; the leading axes index frequencies,
    transmits, right-hand sides or components), rows whose norm is below
    `row_floor` times the largest row norm (or below `abs_floor`) being
    measured against that floor, and
  - the element-wise max |a - b| over max |b| (or `abs_floor`),
so that one wrong field, one wrong transmit row of the data or one wrong grid
point cannot hide inside a norm over the whole output. With rows=False only
the element-wise measure is taken (spectra, FFT outputs, whose rows differ in
magnitude by orders).
"""
import numpy as np


def _np(x):
    try:
        import torch
        if torch.is_tensor(x):
            return x.detach().cpu().numpy()
    except ImportError:  # pragma: no cover
        pass
    return np.asarray(x)


def strict_err(a, b, rows=True, row_floor=1e-6, abs_floor=0.0):
    a = _np(a)
    b = _np(b)
    if a.shape != b.shape:
        raise ValueError(f"shape mismatch {a.shape} vs {b.shape}")
    if a.size == 0:
        return 0.0
    d = np.abs(a - b)
    el = float(d.max() / max(np.abs(b).max(), abs_floor, 1e-300))
    if not rows or a.ndim == 0:
        return el
    A = (a - b).reshape(-1, a.shape[-1])
    Bm = b.reshape(-1, b.shape[-1])
    rn = np.linalg.norm(Bm, axis=1)
    en = np.linalg.norm(A, axis=1)
    floor = max(rn.max() * row_floor, abs_floor, 1e-300)
    row = float((en / np.maximum(rn, floor)).max())
    return max(row, el)


def field_err(a, b):
    """max over fields (leading axes) of ||a - b|| / ||b|| over the grid: the
    field error of the mixed-precision bar."""
    a = _np(a)
    b = _np(b)
    A = (a - b).reshape(-1, a.shape[-1])
    Bm = b.reshape(-1, b.shape[-1])
    return float((np.linalg.norm(A, axis=1) / np.maximum(np.linalg.norm(Bm, axis=1), 1e-300)).max())
