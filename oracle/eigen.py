"""FP64 oracle of the one-group k-eigenvalue power iteration.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU-baseline leg).

Section 5.2, Eq. 26: the fixed source of Eq. 12 is replaced by the fission
emission nu*sigma_f*phi/k (per unit weight in this library's normalisation,
where the weights sum to 1).  Appendix A2 (Eq. A1-A4) solves it with two
nested loops:
  * inner M: the fixed-source problem with the current fission source,
    iterated to convergence (here the FP64 source iteration of ``si1d`` /
    ``si2d``, warm-started from the current eigenfunction), or, in the
    neural-operator variants (Eq. A5, A7-A8), one network application (SP)
    or one network application and one sweep (CP);
  * outer P: new eigenvalue from the fission-production ratio and
    normalisation of the eigenfunction, then a new fission source.

Update P (the normalisation condition of Appendix A2):
    F(phi)   = sum_cells nu_sigma_f * phi * V
    k_new    = k * F(phi_half) / F(phi)
    phi_new  = phi_half / F(phi_half)          (so that F(phi_new) = 1)
Stopping rule (section 5.2 applies one tolerance to k and to phi):
    |k_new - k| / k_new < tol_k  and
    max|phi_new - phi| / max|phi_new| < tol_phi.
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from . import si1d, si2d


class EigenResult:
    def __init__(self, k, phi, outer, inner, dk, dphi, converged, k_hist):
        self.k = k
        self.phi = phi
        self.outer = outer
        self.inner = inner
        self.dk = dk
        self.dphi = dphi
        self.converged = converged
        self.k_history = k_hist


def fission_production(nu_sigma_f, phi, vol):
    """F(phi) = sum nu_sigma_f * phi * V over the cells (FP64)."""
    return float(np.sum(np.asarray(nu_sigma_f, float) * np.asarray(phi, float)) * vol)


def power_iteration(inner: Callable[[np.ndarray, np.ndarray], tuple],
                    nu_sigma_f, vol, phi0=None, k0=1.0, tol_k=1e-10,
                    tol_phi=1e-10, max_outer=10000) -> EigenResult:
    """Outer loop P around a caller-given inner solve (Appendix A2).

    inner(S, phi_warm, k) -> (phi_half, inner_iterations) solves the
    fixed-source problem with isotropic source S = nu_sigma_f phi_warm / k
    from the warm start phi_warm.  phi0 = None starts from a flat flux."""
    nsf = np.asarray(nu_sigma_f, float)
    phi = np.ones_like(nsf) if phi0 is None else np.array(phi0, float)
    F = fission_production(nsf, phi, vol)
    if not F > 0:
        raise ValueError("the initial flux produces no fissions")
    phi = phi / F
    k = float(k0)
    inner_total = 0
    hist = []
    dk = dphi = np.inf
    for n in range(1, max_outer + 1):
        S = nsf * phi / k                          # Eq. 26 fission emission
        phi_half, it = inner(S, phi, k)            # Eq. A2
        inner_total += it
        F_half = fission_production(nsf, phi_half, vol)
        F_old = fission_production(nsf, phi, vol)
        k_new = k * F_half / F_old                 # Eq. A3: eigenvalue
        phi_new = phi_half / F_half                # Eq. A3: normalisation
        dk = abs(k_new - k) / abs(k_new)
        dphi = np.max(np.abs(phi_new - phi)) / np.max(np.abs(phi_new))
        k, phi = k_new, phi_new
        hist.append(k)
        if dk < tol_k and dphi < tol_phi:
            return EigenResult(k, phi, n, inner_total, dk, dphi, True, hist)
    return EigenResult(k, phi, max_outer, inner_total, dk, dphi, False, hist)


def si_inner(inst, quad, tol):
    """Inner M for an ``inputs.Instance``: FP64 source iteration to ``tol``
    (max-norm in 1-D, relative L2 in 2-D), warm-started."""
    if inst.dim == 1:
        def inner(S, phi, k):
            r = si1d(inst.nx, inst.lx, quad.mu, quad.w, inst.sigma_t,
                     inst.sigma_s, S, bc=inst.bc[:2], phi0=phi, tol=tol,
                     norm="max")
            return r.phi, r.iterations
    else:
        def inner(S, phi, k):
            r = si2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta,
                     quad.w, inst.sigma_t, inst.sigma_s, S, bc=inst.bc,
                     phi0=phi, tol=tol, norm="l2")
            return r.phi, r.iterations
    return inner


def cell_volume(inst) -> float:
    if inst.dim == 1:
        return inst.lx / inst.nx
    return (inst.lx / inst.nx) * (inst.ly / inst.ny)


def solve_eigen(inst, quad, nu_sigma_f, tol_inner=1e-12, tol_k=1e-10,
                tol_phi=1e-10, phi0=None, k0=1.0, max_outer=10000) -> EigenResult:
    """Model-based k-eigenvalue solve of one instance (its ``source`` field
    is not used; the fission emission replaces it)."""
    nsf = np.asarray(nu_sigma_f, float).reshape(np.shape(inst.sigma_t))
    return power_iteration(si_inner(inst, quad, tol_inner), nsf,
                           cell_volume(inst), phi0=phi0, k0=k0, tol_k=tol_k,
                           tol_phi=tol_phi, max_outer=max_outer)


# ------------------------------------------------ neural-operator variants --
# Appendix A2 (i)-(ii).  linv_star(S) -> phi is the inverse transport operator
# at the training parameters p* (the network, wrapped by
# recast.network_inner, or an exact solve for the checks); the parameter
# deviation enters as the recast source (sigma_a* - sigma_a) phi of Eq. 24.

def sp_inner(linv_star, sigma_a, sigma_a_star):
    """Simple preconditioning, Eq. A5: the inner solve is one application of
    linv_star to the fission source plus the recast term of the current
    iterate."""
    sa = np.asarray(sigma_a, float)

    def inner(S, phi, k):
        return linv_star(S + (sigma_a_star - sa) * phi), 1
    return inner


def cp_inner(linv_star, sigma_a, sigma_a_star, sweep, sigma_s, nu_sigma_f):
    """Constrained preconditioning, Eq. A7-A8: the prediction u of Eq. A7,
    then one transport sweep (one application of the source-iteration
    operator) of the emission sigma_s u + nu_sigma_f u / k, the fission
    term taken from u with the current eigenvalue."""
    sa = np.asarray(sigma_a, float)
    ss = np.asarray(sigma_s, float)
    nsf = np.asarray(nu_sigma_f, float)

    def inner(S, phi, k):
        u = linv_star(S + (sigma_a_star - sa) * phi)
        return sweep(ss * u + nsf * u / k), 1
    return inner


def solve_eigen_no(inst, quad, nu_sigma_f, linv_star, sigma_a_star, variant,
                   tol_k=1e-10, tol_phi=1e-10, phi0=None, k0=1.0,
                   max_outer=10000) -> EigenResult:
    """The neural-operator outer loop of one 2-D instance (variant "sp" or
    "cp"); its result is the starting pair of the model-based refinement
    (Eq. A6)."""
    from . import sweep2d
    nsf = np.asarray(nu_sigma_f, float).reshape(inst.ny, inst.nx)
    sa = np.asarray(inst.sigma_t, float) - np.asarray(inst.sigma_s, float)
    if variant == "sp":
        inner = sp_inner(linv_star, sa, sigma_a_star)
    elif variant == "cp":
        def sweep(Q):
            return sweep2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta,
                           quad.w, inst.sigma_t, Q, bc=inst.bc)
        inner = cp_inner(linv_star, sa, sigma_a_star, sweep, inst.sigma_s, nsf)
    else:
        raise ValueError(variant)
    return power_iteration(inner, nsf, cell_volume(inst), phi0=phi0, k0=k0,
                           tol_k=tol_k, tol_phi=tol_phi, max_outer=max_outer)


# ------------------------------------------------------------ multigroup ----
# Section 5.3, Eq. 27-29: G groups with downscatter only (no upscatter),
# isotropic scattering, fission spectrum chi.  Group g sees the emission
#   sigma_s^{g->g} phi_g + sum_{h<g} sigma_s^{h->g} phi_h
#     + chi_g / k * sum_h nu_sigma_f_h phi_h .
# Inner M: one pass over the groups in order (Gauss-Seidel in energy), each
# group's source iteration run to tol_inner with the fission density of the
# previous outer iterate and the downscatter of the groups already solved in
# this pass; without upscatter one pass solves the fixed-source problem.
# Outer P as in the one-group loop with F(phi) = sum_g sum_cells
# nu_sigma_f_g phi_g V and the max-norm change taken over all groups.

def fission_production_mg(nu_sigma_f, phi, vol):
    return float(sum(np.sum(np.asarray(f, float) * np.asarray(p, float))
                     for f, p in zip(nu_sigma_f, phi)) * vol)


def solve_eigen_mg(inst, quad, sigma_t, sigma_s, nu_sigma_f, chi, tol_inner=1e-12,
                   tol_k=1e-10, tol_phi=1e-10, phi0=None, k0=1.0,
                   max_outer=10000) -> EigenResult:
    """inst gives the geometry (grid, extents, faces); sigma_t[g],
    nu_sigma_f[g] fields; sigma_s[g][h] the g -> h field (None = zero),
    upscatter (h < g) must be None; chi[g] scalars.  phi is (G, ny, nx)."""
    G = len(sigma_t)
    shape = np.shape(inst.sigma_t)
    st = [np.asarray(a, float).reshape(shape) for a in sigma_t]
    nsf = [np.asarray(a, float).reshape(shape) for a in nu_sigma_f]
    ss = [[None if sigma_s[g][h] is None else np.asarray(sigma_s[g][h], float).reshape(shape)
           for h in range(G)] for g in range(G)]
    for g in range(G):
        for h in range(g):
            if ss[g][h] is not None:
                raise ValueError("upscatter is not modelled")
    vol = cell_volume(inst)
    phi = np.ones((G,) + shape) if phi0 is None else np.array(phi0, float).reshape((G,) + shape)
    F = fission_production_mg(nsf, phi, vol)
    if not F > 0:
        raise ValueError("the initial flux produces no fissions")
    phi = phi / F
    k = float(k0)
    inner_total, hist = 0, []
    dk = dphi = np.inf
    zero = np.zeros(shape)

    def group_solve(g, q, warm):
        sg = ss[g][g] if ss[g][g] is not None else zero
        if inst.dim == 1:
            r = si1d(inst.nx, inst.lx, quad.mu, quad.w, st[g], sg, q, bc=inst.bc[:2],
                     phi0=warm, tol=tol_inner, norm="max")
        else:
            r = si2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta, quad.w,
                     st[g], sg, q, bc=inst.bc, phi0=warm, tol=tol_inner, norm="l2")
        return r.phi.reshape(shape), r.iterations

    for n in range(1, max_outer + 1):
        fis = sum(f * p for f, p in zip(nsf, phi)) / k        # Eq. 27-29 fission density
        half = np.zeros_like(phi)
        for g in range(G):
            q = chi[g] * fis
            for h in range(g):
                if ss[h][g] is not None:
                    q = q + ss[h][g] * half[h]                 # downscatter h -> g
            half[g], it = group_solve(g, q, phi[g])
            inner_total += it
        F_half = fission_production_mg(nsf, half, vol)
        F_old = fission_production_mg(nsf, phi, vol)
        k_new = k * F_half / F_old
        phi_new = half / F_half
        dk = abs(k_new - k) / abs(k_new)
        dphi = np.max(np.abs(phi_new - phi)) / np.max(np.abs(phi_new))
        k, phi = k_new, phi_new
        hist.append(k)
        if dk < tol_k and dphi < tol_phi:
            return EigenResult(k, phi, n, inner_total, dk, dphi, True, hist)
    return EigenResult(k, phi, max_outer, inner_total, dk, dphi, False, hist)
