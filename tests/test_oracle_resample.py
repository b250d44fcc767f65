"""Pins of the oracle's grid transfers (block average to the network grid,
bilinear interpolation back, cell-centred with clamped edges)."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import resample as RS


@pytest.mark.parametrize("n,f", [(8, 4), (6, 2), (5, 3)])
def test_block_average_keeps_integrals_and_linear_fields(n, f):
    rng = np.random.Generator(np.random.PCG64(n * 10 + f))
    fine = rng.uniform(-1.0, 3.0, (n * f, n * f))
    h = 10.0 / (n * f)
    c = RS.block_average(fine, f)
    assert c.shape == (n, n)
    assert abs(c.sum() * (f * h) ** 2 - fine.sum() * h * h) < 1e-12 * np.abs(fine).sum() * h * h
    # every coarse value is the integral of its block over the block's area
    for J, I in ((0, 0), (n - 1, 1), (n // 2, n - 1)):
        blk = fine[J * f:(J + 1) * f, I * f:(I + 1) * f]
        assert abs(c[J, I] - blk.sum() * h * h / (f * h) ** 2) < 1e-14 * np.abs(blk).sum()
    # a linear function sampled at fine centres averages to its value at
    # the coarse centres
    xf = (np.arange(n * f) + 0.5) * h
    xc = (np.arange(n) + 0.5) * f * h
    lin = lambda x, y: 0.3 + 1.7 * x - 0.4 * y
    c = RS.block_average(lin(xf[None, :], xf[:, None]), f)
    assert np.abs(c - lin(xc[None, :], xc[:, None])).max() < 1e-12


@pytest.mark.parametrize("n,f", [(8, 4), (7, 2), (4, 3)])
def test_bilinear_reproduces_bilinear_functions(n, f):
    """g(x, y) = a + b x + c y + d x y sampled at coarse centres comes back
    exactly at every fine centre inside the span of the coarse centres, and
    at the clamped point (nearest point of that span) outside it."""
    g = lambda x, y: 0.5 - 0.25 * x + 2.0 * y + 0.75 * x * y
    xc = np.arange(n) + 0.5                 # coarse centres, coarse-cell units
    xf = (np.arange(n * f) + 0.5) / f       # fine centres
    coarse = g(xc[None, :], xc[:, None])
    up = RS.bilinear_up(coarse, f)
    xcl = np.clip(xf, xc[0], xc[-1])
    want = g(xcl[None, :], xcl[:, None])
    assert np.abs(up - want).max() < 1e-12 * np.abs(want).max()
    inside = (xf >= xc[0]) & (xf <= xc[-1])
    assert inside.sum() == n * f - 2 * (f // 2)
    xi = xf[inside]
    assert np.abs(up[np.ix_(inside, inside)] - g(xi[None, :], xi[:, None])).max() < 1e-12 * 20


@pytest.mark.parametrize("n,f", [(8, 4), (6, 2)])
def test_bilinear_matches_library_interpolator(n, f):
    """Random coarse data: the same values as scipy's linear
    RegularGridInterpolator at the (clamped) fine centres."""
    rng = np.random.Generator(np.random.PCG64(3 + n))
    coarse = rng.uniform(0.0, 1.0, (n, n))
    xc = np.arange(n) + 0.5
    xf = np.clip((np.arange(n * f) + 0.5) / f, xc[0], xc[-1])
    interp = RegularGridInterpolator((xc, xc), coarse, method="linear")
    Y, X = np.meshgrid(xf, xf, indexing="ij")
    want = interp(np.stack([Y.ravel(), X.ravel()], axis=1)).reshape(n * f, n * f)
    assert np.abs(RS.bilinear_up(coarse, f) - want).max() < 1e-14


def test_constant_round_trip_and_factor_one():
    c = np.full((4, 4), 2.5)
    assert np.abs(RS.bilinear_up(c, 4) - 2.5).max() == 0.0
    rng = np.random.Generator(np.random.PCG64(9))
    a = rng.uniform(0.0, 1.0, (6, 6))
    assert np.array_equal(RS.block_average(a, 1), a)
    assert np.abs(RS.bilinear_up(a, 1) - a).max() == 0.0
    assert np.abs(RS.block_average(RS.bilinear_up(np.full((3, 3), 1.25), 2), 2) - 1.25).max() < 1e-15
