"""Equation-recast loop (arXiv 2509.01416 Eq. 7/8 in general form, Eq. 24 for
the transport equation), FP64.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

With p = p* + dp the transport operator is split as L(p) = L(p*) + dL(dp) and
the deviation moved to the source (Eq. 6b-7a).  Under the isotropic
approximation of Eq. 23 the scalar-flux update of Eq. 24 reads

    phi^(k+1) = Linv(p*) [ S + ((sigma_s - sigma_s*) - (sigma_t - sigma_t*)) phi^(k) ]
              = Linv(p*) [ S + (sigma_a* - sigma_a) phi^(k) ],

where Linv(p*) is either the pretrained network or, for the closed-form
check, the exact transport solution operator at the training parameters.

Controller readings (the paper gives none of these): phi^(0) = 0; stop when
||phi^(k+1) - phi^(k)||_2 / ||phi^(k+1)||_2 < tol (default 1e-4, the paper's
universal tolerance) or after max_iter (default 30) updates; declare
divergence when the change is non-finite, or when the absolute change
||phi^(k+1) - phi^(k)||_2 has grown for three consecutive updates and exceeds
the first update's (a geometric divergence keeps the relative change near the
constant 1 - 1/gain, so the absolute change is the one that grows); and
accept as converged a loop that has stalled close to the tolerance: the
relative change is below 10 tol but no lower than 0.9 times its value three
updates earlier (a network evaluated in BF16 has a rounding floor of its
own, about 3e-4 to 2e-3 relative, that a tight tolerance cannot pass; the
guess is then as good as the network makes it).
"""
from __future__ import annotations

from typing import Callable

import numpy as np

CONVERGED = 0
NOT_CONVERGED = 1
DIVERGED = 2


def recast_source(S, sigma_a, sigma_a_star, phi):
    """Eq. 24 right-hand side: S + (sigma_a* - sigma_a) phi."""
    return S + (sigma_a_star - sigma_a) * phi


STALL_FACTOR = 10.0     # stall only below this multiple of tol
STALL_DROP = 0.9        # ... when the change fell by less than this
STALL_LAG = 3           # ... over this many updates


def recast_loop(S: np.ndarray, sigma_a: np.ndarray, sigma_a_star: float,
                inner: Callable[[np.ndarray], np.ndarray], tol: float = 1e-4,
                max_iter: int = 30, grow_limit: int = 3):
    """Iterate Eq. 24 with the inner operator `inner` (S_eff -> phi).

    Returns (phi, status, iterations, history of change norms)."""
    phi = np.zeros_like(S, dtype=np.float64)
    hist = []
    absd = []
    grow = 0
    for k in range(max_iter):
        new = inner(recast_source(S, sigma_a, sigma_a_star, phi))
        num = np.sqrt(np.sum((new - phi) ** 2))
        den = np.sqrt(np.sum(new * new))
        d = num / den if den > 0 else (0.0 if num == 0 else np.inf)
        hist.append(d)
        absd.append(num)
        phi = new
        if not (np.isfinite(d) and np.isfinite(num)):
            return np.zeros_like(phi), DIVERGED, k + 1, hist
        if d < tol:
            return phi, CONVERGED, k + 1, hist
        if (k >= STALL_LAG and d < STALL_FACTOR * tol
                and d > STALL_DROP * hist[k - STALL_LAG]):
            return phi, CONVERGED, k + 1, hist
        grow = grow + 1 if (k >= 1 and num > absd[-2]) else 0
        if grow >= grow_limit and num > absd[0]:
            return np.zeros_like(phi), DIVERGED, k + 1, hist
    return phi, NOT_CONVERGED, max_iter, hist


def network_inner(forward: Callable[[np.ndarray], np.ndarray],
                  sigma_a_star: float):
    """Wrap a network trained on (S / s, sigma_a* phi / s) pairs, with
    s = mean |S|, as an operator S_eff -> phi.  Exact for the exact
    operator by linearity of Linv(p*)."""
    def inner(S_eff):
        s = np.mean(np.abs(S_eff))
        if s == 0.0:
            return np.zeros_like(S_eff)
        return forward(S_eff / s) * s / sigma_a_star
    return inner
