"""Grid transfers of the recast guess between a solver grid and the network
grid, FP64.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The operator network is trained on one grid (64 x 64 cells on the 10 x 10
domain); a problem on an n f x n f grid of the same domain runs the
equation-recast loop of Eq. 24 on the network grid and hands the guess back
to its own grid.  The paper works on one grid throughout and says nothing
about this; the readings are:

  * fine -> coarse: the mean over each f x f block of fine cells.  On uniform
    cells that is the cell average of the piecewise-constant fine field over
    the coarse cell, so integrals over the domain are kept exactly;
  * coarse -> fine: bilinear interpolation between coarse cell centres, the
    value at each fine cell centre; fine centres closer to the boundary than
    the outermost coarse centres take the value at the nearest point of the
    rectangle spanned by the coarse centres (clamped edges).

Coordinates are in units of coarse cells: coarse centre I sits at I + 1/2,
fine centre i at (i + 1/2) / f.
"""
from __future__ import annotations

import numpy as np


def block_average(a: np.ndarray, f: int) -> np.ndarray:
    """Mean over f x f blocks of a (ny, nx) field with f | nx, f | ny."""
    a = np.asarray(a, dtype=np.float64)
    ny, nx = a.shape
    if nx % f or ny % f:
        raise ValueError("the block size must divide both grid sides")
    out = np.zeros((ny // f, nx // f))
    for J in range(ny // f):
        for I in range(nx // f):
            out[J, I] = a[J * f:(J + 1) * f, I * f:(I + 1) * f].sum() / (f * f)
    return out


def _axis_weights(n: int, f: int):
    """For each of the n f fine centres along one axis: the two coarse
    centres that bracket it and the weight of the second one."""
    lo = np.zeros(n * f, dtype=np.int64)
    hi = np.zeros(n * f, dtype=np.int64)
    t = np.zeros(n * f)
    for i in range(n * f):
        # fine centre in the index space of coarse centres (centre I at I)
        p = (i + 0.5) / f - 0.5
        p = min(max(p, 0.0), float(n - 1))   # clamped to the centres' span
        I0 = min(int(np.floor(p)), n - 2) if n > 1 else 0
        lo[i] = I0
        hi[i] = min(I0 + 1, n - 1)
        t[i] = p - I0
    return lo, hi, t


def bilinear_up(c: np.ndarray, f: int) -> np.ndarray:
    """Bilinear interpolation of a coarse (ny, nx) cell-centred field onto
    the f-times finer grid (clamped edges)."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    xl, xh, tx = _axis_weights(nx, f)
    yl, yh, ty = _axis_weights(ny, f)
    out = np.zeros((ny * f, nx * f))
    for j in range(ny * f):
        for i in range(nx * f):
            v00 = c[yl[j], xl[i]]
            v01 = c[yl[j], xh[i]]
            v10 = c[yh[j], xl[i]]
            v11 = c[yh[j], xh[i]]
            out[j, i] = ((1 - ty[j]) * ((1 - tx[i]) * v00 + tx[i] * v01)
                         + ty[j] * ((1 - tx[i]) * v10 + tx[i] * v11))
    return out
