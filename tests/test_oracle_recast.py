"""Closed-form pins of the recast loop (Eq. 24) with the exact operator.

With Linv(p*) the exact transport solution operator at (sigma_t*, sigma_s*),
the fixed point of phi = Linv(p*)[S + (sigma_a* - sigma_a) phi] solves
transport with sigma_t* in the streaming/removal term and scattering
sigma_t* - sigma_a(x): the true absorption but the training total cross
section.  It is the true solution when sigma_t == sigma_t*.
"""
import numpy as np

import oracle
from oracle import recast as RC
from paper_2509_01416_amd import inputs as I


def _exact_inner(n, q, st_star, ss_star):
    st = np.full((n, n), st_star)
    ss = np.full((n, n), ss_star)

    def inner(S):
        return oracle.si2d(n, n, 10.0, 10.0, q.mu, q.eta, q.w, st, ss, S,
                           tol=1e-14).phi
    return inner


def test_recast_fixed_point_closed_form():
    n = 10
    q = I.level_symmetric_2d(4)
    st_star, ss_star = 1.0, 0.8
    sa_star = st_star - ss_star
    st = I.sinusoid_field(n, n, 10.0, 10.0, 1.0, 0.3)
    sa = I.sinusoid_field(n, n, 10.0, 10.0, 0.2, 0.08, "cos")
    S = I.grf_2d(n, 10.0, seed=77)
    phi, status, k, hist = RC.recast_loop(S, sa, sa_star,
                                          _exact_inner(n, q, st_star, ss_star),
                                          tol=1e-12, max_iter=400)
    assert status == RC.CONVERGED
    closed = oracle.si2d(n, n, 10.0, 10.0, q.mu, q.eta, q.w,
                         np.full((n, n), st_star), st_star - sa, S,
                         tol=1e-14).phi
    assert np.abs(phi - closed).max() < 1e-9 * closed.max()
    truth = oracle.si2d(n, n, 10.0, 10.0, q.mu, q.eta, q.w, st, st - sa, S,
                        tol=1e-14).phi
    # not the truth: the isotropic approximation of Eq. 23 is not exact here
    assert np.abs(phi - truth).max() > 1e-4 * truth.max()


def test_recast_exact_when_total_xs_matches():
    n = 8
    q = I.level_symmetric_2d(4)
    st_star, ss_star = 1.0, 0.8
    sa = np.full((n, n), 0.2) + 0.1 * np.random.Generator(
        np.random.PCG64(4)).uniform(-1, 1, (n, n))
    S = I.grf_2d(n, 10.0, seed=78)
    phi, status, k, _ = RC.recast_loop(S, sa, 0.2,
                                       _exact_inner(n, q, st_star, ss_star),
                                       tol=1e-12, max_iter=400)
    assert status == RC.CONVERGED
    truth = oracle.si2d(n, n, 10.0, 10.0, q.mu, q.eta, q.w,
                        np.full((n, n), st_star), st_star - sa, S,
                        tol=1e-14).phi
    assert np.abs(phi - truth).max() < 1e-9 * truth.max()


def test_recast_divergence_guard():
    """A scaled-identity inner operator with gain > 1 grows every update."""
    S = np.ones((4, 4))
    sa = np.full((4, 4), -0.2)        # sigma_a* - sigma_a = 0.4
    phi, status, k, hist = RC.recast_loop(S, sa, 0.2, lambda s: 3.0 * s,
                                          tol=1e-6, max_iter=50)
    assert status == RC.DIVERGED
    assert k <= 6 and np.all(phi == 0)


def test_recast_contraction_rate():
    """inner = c * identity: phi_k = c S sum_{j<k} (c d)^j, change norm ratio
    equals c d."""
    c, d = 2.0, 0.25
    S = np.full((3, 3), 1.0)
    phi, status, k, hist = RC.recast_loop(S, np.full((3, 3), 0.0), d,
                                          lambda s: c * s, tol=1e-10,
                                          max_iter=200)
    assert status == RC.CONVERGED
    assert abs(phi[0, 0] - c / (1 - c * d)) < 1e-9
    ratios = [hist[i + 1] / hist[i] for i in range(2, 8)]
    # relative change ||phi_{k+1}-phi_k|| / ||phi_{k+1}||; tends to (c d)
    assert abs(ratios[-1] - c * d) < 1e-3


def test_recast_stall_rule():
    """A pointwise operator with a rounding-like floor (a fixed pattern of
    relative size 2e-3 flipping sign every update) stalls with a change near
    4e-3: below 10 tol at tol 1e-3, so the loop stops as converged once the
    change has not fallen by 10 % over three updates; at tol 1e-4 the floor
    lies above 10 tol and the loop runs to max_iter.  A clean contraction at
    rate 0.95 (change falling 14 % per three updates) is never stopped by
    the rule and reaches the tolerance."""
    n = 6
    S = np.linspace(1.0, 2.0, n * n).reshape(n, n)
    sa = np.full((n, n), 0.1)
    pattern = np.where(np.arange(n * n).reshape(n, n) % 2 == 0, 1.0, -1.0)
    calls = []

    def noisy(s):
        calls.append(1)
        sign = 1.0 if len(calls) % 2 else -1.0
        return (s / 0.2) * (1.0 + 2e-3 * sign * pattern)
    phi, status, k, hist = RC.recast_loop(S, sa, 0.2, noisy, tol=1e-3, max_iter=30)
    assert status == RC.CONVERGED and hist[-1] > 1e-3 and k < 30
    assert hist[-1] > RC.STALL_DROP * hist[-1 - RC.STALL_LAG]
    calls.clear()
    _, status, k, hist = RC.recast_loop(S, sa, 0.2, noisy, tol=1e-4, max_iter=30)
    assert status == RC.NOT_CONVERGED and k == 30
    # contraction at rate 0.95: sigma_a* - sigma_a = 0.95 sigma_a* for the
    # exact pointwise operator s / sigma_a*
    _, status, k, hist = RC.recast_loop(S, np.full((n, n), 0.01), 0.2, lambda s: s / 0.2,
                                        tol=1e-3, max_iter=400)
    rates = [hist[i + 1] / hist[i] for i in range(5, len(hist) - 1)]
    assert status == RC.CONVERGED and hist[-1] < 1e-3
    assert max(rates) < 0.96
