"""Pins of the oracle's linearly anisotropic (P1) scattering, section 5.1
Eq. 25: the emission of direction m gains 3 sigma_s1 Omega_m . J.

  * source iteration reaches the direct solve of the coupled DD system with
    the P1 coupling written out (1-D slabs and small x-y grids, vacuum and
    reflective faces);
  * one sweep with anisotropic emission fields equals the direct solve of
    that one sweep, and the current it returns equals sum_m w_m Omega_m psi_m
    of the direct solve;
  * the infinite medium keeps phi = q / sigma_a (an isotropic flux carries
    no current, so the P1 term vanishes);
  * sigma_s1 = 0 gives the isotropic answer bit for bit;
  * the P1 term changes the answer (a check that it is not dropped)."""
import numpy as np
import pytest

import oracle
from dd_direct import solve_1d, solve_2d
from paper_2509_01416_amd import inputs as I


def _slab(n, seed, s1):
    rng = np.random.Generator(np.random.PCG64(seed))
    st = rng.uniform(0.8, 1.6, n)
    ss = st * rng.uniform(0.4, 0.8, n)
    return st, ss, np.full(n, s1), rng.uniform(0.2, 1.2, n)


@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_si1d_p1_matches_direct(bc):
    q = I.gauss_legendre(8)
    n, L = 30, 6.0
    st, ss, s1, src = _slab(n, 5, 0.3)
    ref = solve_1d(n, L, q.mu, q.w, st, ss, src, bc=bc, sigma_s1=s1)
    r = oracle.si1d(n, L, q.mu, q.w, st, ss, src, bc=bc, tol=1e-14, sigma_s1=s1)
    assert r.status == oracle.OK
    assert np.abs(r.phi - ref).max() < 1e-11 * np.abs(ref).max()
    iso = solve_1d(n, L, q.mu, q.w, st, ss, src, bc=bc)
    assert np.abs(iso - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 0, 1, 0)])
def test_si2d_p1_matches_direct(bc):
    q = I.level_symmetric_2d(4)
    inst = I.random_instance(6, 5, seed=12, lx=3.0, ly=2.5, c_range=(0.4, 0.8), bc=bc)
    s1 = 0.25 * inst.sigma_s
    ref = solve_2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t,
                   inst.sigma_s, inst.source, bc, sigma_s1=s1)
    r = oracle.si2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t,
                    inst.sigma_s, inst.source, bc=bc, tol=1e-14, sigma_s1=s1)
    assert r.status == oracle.OK
    assert np.abs(r.phi - ref).max() < 1e-11 * np.abs(ref).max()
    iso = solve_2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t,
                   inst.sigma_s, inst.source, bc)
    assert np.abs(iso - ref).max() > 1e-3 * np.abs(ref).max()


def test_sweep2d_anisotropic_emission_and_current():
    q = I.level_symmetric_2d(4)
    inst = I.random_instance(5, 7, seed=4, lx=2.0, ly=3.0)
    rng = np.random.Generator(np.random.PCG64(8))
    Q = rng.uniform(0.5, 1.5, (7, 5))
    ex = rng.uniform(-0.3, 0.3, (7, 5))
    ey = rng.uniform(-0.3, 0.3, (7, 5))
    per_dir = Q[None] + q.mu[:, None, None] * ex[None] + q.eta[:, None, None] * ey[None]
    ref, (jx_ref, jy_ref) = solve_2d(5, 7, 2.0, 3.0, q.mu, q.eta, q.w, inst.sigma_t,
                                     0 * inst.sigma_s, per_dir, (0, 0, 0, 0), coupled=False,
                                     return_current=True)
    phi, (jx, jy) = oracle.sweep2d(5, 7, 2.0, 3.0, q.mu, q.eta, q.w, inst.sigma_t, Q,
                                   ex=ex, ey=ey, return_current=True)
    sc = np.abs(ref).max()
    assert np.abs(phi - ref).max() < 1e-12 * sc
    assert np.abs(jx - jx_ref).max() < 1e-12 * sc
    assert np.abs(jy - jy_ref).max() < 1e-12 * sc


def test_sweep1d_anisotropic_emission_and_current():
    q = I.gauss_legendre(6)
    n, L = 9, 2.0
    st, _, _, Q = _slab(n, 3, 0.0)
    ex = np.linspace(-0.2, 0.3, n)
    # the same sweep as a 2-D problem of one row between reflective y faces
    # would need eta; instead: each direction's slab recurrence by hand
    phi, jx = oracle.sweep1d(n, L, q.mu, q.w, st, Q, ex=ex, return_current=True)
    dx = L / n
    want_phi, want_j = np.zeros(n), np.zeros(n)
    for m in range(len(q.mu)):
        a = 2 * abs(q.mu[m]) / dx
        cells = range(n) if q.mu[m] > 0 else range(n - 1, -1, -1)
        inflow = 0.0
        for i in cells:
            psi = (Q[i] + q.mu[m] * ex[i] + a * inflow) / (st[i] + a)
            inflow = 2 * psi - inflow
            want_phi[i] += q.w[m] * psi
            want_j[i] += q.w[m] * q.mu[m] * psi
    assert np.abs(phi - want_phi).max() < 1e-14 * np.abs(want_phi).max()
    assert np.abs(jx - want_j).max() < 1e-14 * np.abs(want_phi).max()


def test_infinite_medium_with_p1():
    q = I.level_symmetric_2d(4)
    kappa = 0.7
    rng = np.random.Generator(np.random.PCG64(2))
    st = rng.uniform(1.0, 2.0, (4, 4))
    ss = 0.6 * st
    r = oracle.si2d(4, 4, 1.0, 1.0, q.mu, q.eta, q.w, st, ss, kappa * (st - ss),
                    bc=(1, 1, 1, 1), tol=1e-14, sigma_s1=0.2 * st)
    assert np.abs(r.phi - kappa).max() < 1e-12


def test_zero_p1_is_isotropic_bit_for_bit():
    q = I.level_symmetric_2d(4)
    inst = I.random_instance(7, 6, seed=21)
    a = oracle.si2d(7, 6, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t, inst.sigma_s,
                    inst.source, tol=1e-12)
    b = oracle.si2d(7, 6, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t, inst.sigma_s,
                    inst.source, tol=1e-12, sigma_s1=np.zeros((6, 7)))
    assert a.iterations == b.iterations and np.array_equal(a.phi, b.phi)
