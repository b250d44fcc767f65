"""Pins of the oracle's convergence norms and of its error-bound stopping
rule.

The paper quotes only a tolerance for its iterations (section 5.1); the
norms are the library's reading: the relative L2 change, the max relative
change, and the error bound r rho / (1 - rho) of a fixed-point iteration
with observed contraction rate rho = r_l / r_(l-1).  The first two are
pinned by a two-cell slab whose one-sweep answer is worked out by hand; the
error bound by a dense direct solve of a slowly converging problem.
"""
import math

import numpy as np

import oracle
from dd_direct import solve_2d
from paper_2509_01416_amd import inputs as I


def _two_cell_phi():
    """Two cells of width 1, sigma_t = 1, no scattering, q = 1, vacuum,
    S2 Gauss-Legendre (mu = +-1/sqrt 3, weights 1/2 each).  With
    a = 2|mu|/dx = 2/sqrt 3, the direction entering cell 0 gives
    psi_0 = 1/(1+a), leaves it with 2 psi_0, and gives
    psi_1 = (1 + 2a/(1+a))/(1+a) in cell 1; the mirror direction gives the
    same values mirrored, so both cells hold phi = (1+2a)/(1+a)^2."""
    a = 2.0 / math.sqrt(3.0)
    return (1.0 + 2.0 * a) / (1.0 + a) ** 2


def test_change_norms_two_cell_slab_by_hand():
    q = I.gauss_legendre(2)
    st, ss, src = np.ones(2), np.zeros(2), np.ones(2)
    phi = _two_cell_phi()
    u, v = 2.0, 1.5      # the start the single iteration is measured against
    start = np.array([u, v])
    r = oracle.si1d(2, 2.0, q.mu, q.w, st, ss, src, phi0=start, tol=0.0,
                    max_iter=1, norm="l2")
    assert np.abs(r.phi - phi).max() < 1e-15
    l2 = math.sqrt((phi - u) ** 2 + (phi - v) ** 2) / (math.sqrt(2.0) * phi)
    assert abs(r.residual - l2) < 1e-15
    r = oracle.si1d(2, 2.0, q.mu, q.w, st, ss, src, phi0=start, tol=0.0,
                    max_iter=1, norm="max")
    mx = max(abs(phi - u), abs(phi - v)) / phi
    assert abs(r.residual - mx) < 1e-15
    # a denominator taken from the old iterate would give a different value
    assert abs(l2 - math.sqrt((phi - u) ** 2 + (phi - v) ** 2)
               / math.sqrt(u * u + v * v)) > 0.1


def test_change_norm_two_dimensional_matches_slab_definition():
    """The 2-D loop reports the same relative L2 change of one iteration as
    the definition applied to the sweep it performs (start given)."""
    q = I.level_symmetric_2d(4)
    inst = I.random_instance(5, 4, seed=8, lx=2.0, ly=1.5)
    rng = np.random.Generator(np.random.PCG64(1))
    start = rng.uniform(0.5, 1.5, (4, 5))
    r = oracle.si2d(5, 4, 2.0, 1.5, q.mu, q.eta, q.w, inst.sigma_t,
                    inst.sigma_s, inst.source, phi0=start, tol=0.0, max_iter=1)
    one = oracle.sweep2d(5, 4, 2.0, 1.5, q.mu, q.eta, q.w, inst.sigma_t,
                         inst.sigma_s * start + inst.source)
    assert np.abs(r.phi - one).max() < 1e-15 * np.abs(one).max()
    want = np.sqrt(np.sum((one - start) ** 2) / np.sum(one ** 2))
    assert abs(r.residual - want) < 1e-14 * want


def _slow_problem():
    """8 x 8 cells, S4, sigma_t = 1, c = 0.98 and three reflective faces:
    source iteration contracts slowly (rate near 0.95)."""
    q = I.level_symmetric_2d(4)
    inst = I.random_instance(8, 8, seed=17, lx=8.0, ly=8.0, c_range=(0.98, 0.98),
                             st_range=(1.0, 1.0), bc=(1, 1, 1, 0))
    ref = solve_2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w,
                   inst.sigma_t, inst.sigma_s, inst.source, inst.bc)
    return q, inst, ref


def _solve(q, inst, tol, norm):
    return oracle.si2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w,
                       inst.sigma_t, inst.sigma_s, inst.source, bc=inst.bc,
                       tol=tol, norm=norm)


def test_error_bound_rule_meets_its_tolerance():
    """Stopping on r rho/(1 - rho) < tol leaves the iterate within tol of the
    direct solution (relative L2) and not far inside it (the bound is tight
    once the slowest mode dominates); stopping on the plain change at the
    same tol leaves an error far above tol."""
    q, inst, ref = _slow_problem()
    for tol in (1e-5, 1e-7):
        b = _solve(q, inst, tol, "bound")
        e = np.linalg.norm(b.phi - ref) / np.linalg.norm(ref)
        assert b.status == oracle.OK and e <= tol, (tol, e)
        assert e > 0.2 * tol, (tol, e)
        h = b.history
        rho = h[-1] / h[-2]
        assert 0.9 < rho < 1.0
        assert h[-1] * rho / (1 - rho) < tol
        # the previous iteration had not yet met the bound
        rho_p = h[-2] / h[-3]
        assert h[-2] * rho_p / (1 - rho_p) >= tol
        c = _solve(q, inst, tol, "l2")
        ec = np.linalg.norm(c.phi - ref) / np.linalg.norm(ref)
        assert ec > 5 * tol, (tol, ec)


def test_error_bound_rule_exact_fixed_point_and_first_iteration():
    """r = 0 stops at once (the start is the fixed point); otherwise the rule
    needs two change norms, so it never stops on the first iteration."""
    q = I.level_symmetric_2d(4)
    kappa = 1.7
    st = np.full((3, 3), 1.3)
    ss = np.full((3, 3), 0.9)
    r = oracle.si2d(3, 3, 1.0, 1.0, q.mu, q.eta, q.w, st, ss, kappa * (st - ss),
                    bc=(1, 1, 1, 1), phi0=np.full((3, 3), kappa), tol=1e-30,
                    norm="bound")
    assert r.status == oracle.OK and r.iterations == 1 and r.residual == 0.0
    inst = I.random_instance(4, 4, seed=3, c_range=(0.0, 0.0))
    r = oracle.si2d(4, 4, inst.lx, inst.ly, q.mu, q.eta, q.w, inst.sigma_t,
                    inst.sigma_s, inst.source, tol=1e300, norm="bound")
    assert r.iterations >= 2


def test_strided_error_bound_rule():
    """With a stride K the rule tests every K-th iteration on the change over
    K iterations: the stop falls on a multiple of K, the reported change is
    ||phi_l - phi_(l-K)|| / ||phi_l|| of the two iterates, the test at l - K
    had not passed, and the answer lies within tol of the direct solution."""
    q, inst, ref = _slow_problem()
    K = 16
    for tol in (1e-5, 1e-7):
        b = oracle.si2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w,
                        inst.sigma_t, inst.sigma_s, inst.source, bc=inst.bc,
                        tol=tol, norm="bound", stride=K)
        e = np.linalg.norm(b.phi - ref) / np.linalg.norm(ref)
        assert b.status == oracle.OK and b.iterations % K == 0
        assert 0.1 * tol < e <= tol, (tol, e)
        a = oracle.si2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w,
                        inst.sigma_t, inst.sigma_s, inst.source, bc=inst.bc,
                        tol=tol, norm="bound", stride=K, max_iter=b.iterations - K)
        assert a.status == oracle.NOT_CONVERGED
        r = np.linalg.norm(b.phi - a.phi) / np.linalg.norm(b.phi)
        assert abs(b.residual - r) < 1e-12 * r
        # stride 1 is the plain rule, bit for bit
        c1 = oracle.si2d(inst.nx, inst.ny, inst.lx, inst.ly, q.mu, q.eta, q.w,
                         inst.sigma_t, inst.sigma_s, inst.source, bc=inst.bc,
                         tol=tol, norm="bound", stride=1)
        c0 = _solve(q, inst, tol, "bound")
        assert c1.iterations == c0.iterations and np.array_equal(c1.phi, c0.phi)
