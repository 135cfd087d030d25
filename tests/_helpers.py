"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np


def tmunu_rel_err(a, b):
    """max over sites of ||T_a - T_b||_F / ||T_b||_F over the 7 T^{mu nu}
    components (observables 0..6, with T^{tau x} etc. counted twice as the
    symmetric off-diagonal entries)."""
    w = np.array([1, 2, 2, 1, 2, 1, 1.0])[:, None, None]
    d = np.sqrt(np.sum(w * (a[:7] - b[:7]) ** 2, axis=0))
    n = np.sqrt(np.sum(w * b[:7] ** 2, axis=0))
    return float(np.max(d / n))


def patch(arr, cy, cx, r):
    """(..., 2r+1, 2r+1) periodic window of arr (..., ny, nx) centred at (cy, cx)."""
    ny, nx = arr.shape[-2:]
    ys = np.arange(cy - r, cy + r + 1) % ny
    xs = np.arange(cx - r, cx + r + 1) % nx
    return arr[..., ys[:, None], xs[None, :]]
