"""Direct (non-iterative) solve of the diamond-difference S_N equations.

Test helper, independent of the oracle's sweep: it assembles the global linear
system of every cell-centre and face angular flux, with the cell balance,
the two diamond relations and the incoming boundary conditions written as
equations, and solves it with a sparse LU.  Reflective faces are coupled
exactly (not lagged), so a converged source iteration must reach the same
scalar flux.

Equations per direction m and cell (i, j), signed cosines (mu, eta):
    mu (psiX[i+1,j] - psiX[i,j]) / dx + eta (psiY[i,j+1] - psiY[i,j]) / dy
        + sigma_t psiC - [coupled] sigma_s sum_m' w_m' psiC_m'  = rhs
    psiC - (psiX[i+1,j] + psiX[i,j]) / 2 = 0
    psiC - (psiY[i,j+1] + psiY[i,j]) / 2 = 0
Incoming faces: vacuum -> psi = 0; reflective -> psi_m = psi_mirror(m).
With linearly anisotropic scattering (sigma_s1, section 5.1 Eq. 25) the
coupling of direction m to direction k gains 3 sigma_s1 w_k (Omega_m .
Omega_k), the P1 term written out.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _mirror(mu, eta, m, flip_x):
    tm = -mu[m] if flip_x else mu[m]
    te = (eta[m] if flip_x else -eta[m]) if eta is not None else 0.0
    for k in range(len(mu)):
        de = abs(eta[k] - te) if eta is not None else 0.0
        if abs(mu[k] - tm) < 1e-12 and de < 1e-12:
            return k
    raise ValueError("quadrature not reflection symmetric")


def solve_2d(nx, ny, lx, ly, mu, eta, w, sigma_t, sigma_s, rhs, bc,
             coupled=True, sigma_s1=None, return_current=False):
    """Return phi (ny, nx) [and the current (jx, jy)].  coupled=False solves
    one sweep for emission rhs (sigma_s ignored, reflective faces get the
    value 0 instead); rhs may also be given per direction, (M, ny, nx)."""
    M = len(mu)
    dx, dy = lx / nx, ly / ny
    nC = nx * ny
    nX = (nx + 1) * ny
    nY = nx * (ny + 1)
    per = nC + nX + nY
    N = M * per
    st = np.asarray(sigma_t, float).reshape(ny, nx)
    ss = np.asarray(sigma_s, float).reshape(ny, nx)
    s1 = None if sigma_s1 is None else np.asarray(sigma_s1, float).reshape(ny, nx)
    r = np.asarray(rhs, float)
    r = r.reshape(M, ny, nx) if r.size == M * nx * ny else np.broadcast_to(
        r.reshape(ny, nx), (M, ny, nx))

    def C(m, i, j):
        return m * per + j * nx + i

    def X(m, i, j):          # x-face i in [0, nx], row j
        return m * per + nC + j * (nx + 1) + i

    def Y(m, i, j):          # y-face j in [0, ny], column i
        return m * per + nC + nX + j * nx + i

    rows, cols, vals = [], [], []
    b = np.zeros(N)
    eq = 0

    def add(rw, cl, v):
        rows.append(rw)
        cols.append(cl)
        vals.append(v)

    for m in range(M):
        for j in range(ny):
            for i in range(nx):
                add(eq, X(m, i + 1, j), mu[m] / dx)
                add(eq, X(m, i, j), -mu[m] / dx)
                add(eq, Y(m, i, j + 1), eta[m] / dy)
                add(eq, Y(m, i, j), -eta[m] / dy)
                add(eq, C(m, i, j), st[j, i])
                if coupled:
                    for k in range(M):
                        g = ss[j, i]
                        if s1 is not None:
                            g += 3.0 * s1[j, i] * (mu[m] * mu[k] + eta[m] * eta[k])
                        add(eq, C(k, i, j), -g * w[k])
                b[eq] = r[m, j, i]
                eq += 1
                add(eq, C(m, i, j), 1.0)
                add(eq, X(m, i + 1, j), -0.5)
                add(eq, X(m, i, j), -0.5)
                eq += 1
                add(eq, C(m, i, j), 1.0)
                add(eq, Y(m, i, j + 1), -0.5)
                add(eq, Y(m, i, j), -0.5)
                eq += 1
        # incoming x faces
        fin = 0 if mu[m] > 0 else 1
        ib = 0 if mu[m] > 0 else nx
        mx = _mirror(mu, eta, m, True)
        for j in range(ny):
            add(eq, X(m, ib, j), 1.0)
            if bc[fin] == 1 and coupled:
                add(eq, X(mx, ib, j), -1.0)
            eq += 1
        fin = 2 if eta[m] > 0 else 3
        jb = 0 if eta[m] > 0 else ny
        my = _mirror(mu, eta, m, False)
        for i in range(nx):
            add(eq, Y(m, i, jb), 1.0)
            if bc[fin] == 1 and coupled:
                add(eq, Y(my, i, jb), -1.0)
            eq += 1
    assert eq == N
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    x = spla.spsolve(A.tocsc(), b)
    phi = np.zeros((ny, nx))
    jx = np.zeros((ny, nx))
    jy = np.zeros((ny, nx))
    for m in range(M):
        psi = x[m * per:m * per + nC].reshape(ny, nx)
        phi += w[m] * psi
        jx += w[m] * mu[m] * psi
        jy += w[m] * eta[m] * psi
    return (phi, (jx, jy)) if return_current else phi


def solve_1d(nx, lx, mu, w, sigma_t, sigma_s, q, bc=(0, 0), sigma_s1=None):
    """Coupled 1-D DD system (cell and face fluxes of every direction)."""
    M = len(mu)
    dx = lx / nx
    per = nx + nx + 1
    N = M * per
    st = np.asarray(sigma_t, float).reshape(-1)
    ss = np.asarray(sigma_s, float).reshape(-1)
    s1 = None if sigma_s1 is None else np.asarray(sigma_s1, float).reshape(-1)
    qq = np.asarray(q, float).reshape(-1)
    rows, cols, vals = [], [], []
    b = np.zeros(N)
    eq = 0

    def add(rw, cl, v):
        rows.append(rw)
        cols.append(cl)
        vals.append(v)

    for m in range(M):
        C0 = m * per
        F0 = m * per + nx
        for i in range(nx):
            add(eq, F0 + i + 1, mu[m] / dx)
            add(eq, F0 + i, -mu[m] / dx)
            add(eq, C0 + i, st[i])
            for k in range(M):
                g = ss[i] + (0.0 if s1 is None else 3.0 * s1[i] * mu[m] * mu[k])
                add(eq, k * per + i, -g * w[k])
            b[eq] = qq[i]
            eq += 1
            add(eq, C0 + i, 1.0)
            add(eq, F0 + i + 1, -0.5)
            add(eq, F0 + i, -0.5)
            eq += 1
        fin = 0 if mu[m] > 0 else 1
        ib = 0 if mu[m] > 0 else nx
        add(eq, F0 + ib, 1.0)
        if bc[fin] == 1:
            mm = _mirror(mu, None, m, True)
            add(eq, mm * per + nx + ib, -1.0)
        eq += 1
    assert eq == N
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    x = spla.spsolve(A.tocsc(), b)
    phi = np.zeros(nx)
    for m in range(M):
        phi += w[m] * x[m * per:m * per + nx]
    return phi
