"""Pins of the FP64 k-eigenvalue oracle (section 5.2 Eq. 26; Appendix A2).

Each pin stands apart from the oracle's power iteration:
  * the infinite medium (reflective on every face, uniform data), where the
    eigenvalue is nu*sigma_f / sigma_a and the flux is flat;
  * a brute-force eigen-solve on tiny grids: the fixed-source response G of
    the global diamond-difference system (sparse direct solves, one per
    cell, tests/dd_direct.py) gives k as the dominant eigenvalue of
    G diag(nu*sigma_f), with no iteration at all;
  * the eigenvalue printed for eigen Case 1 (Table 7), under the reading
    nu = 3 and vacuum slab faces;
  * linearity: scaling nu*sigma_f by a scales k by a; the limit does not
    depend on the starting flux or eigenvalue;
  * the neural-operator variants SP and CP (Eq. A5, A7-A8): driven by the
    exact p* operator they reach the model-based eigenpair when only
    sigma_s differs from p* (then the recast is exact), and with a
    pointwise linear network SP's eigenvalue has a closed form;
  * three groups (section 5.3, Tables 8-10): the printed model-based k on
    the section 5.1 slab, the infinite-medium k and group spectrum from the
    3 x 3 balance, and a brute-force eigen-solve of the multigroup map.
"""
import numpy as np
import pytest

from dd_direct import solve_1d, solve_2d
from oracle import eigen as E
from paper_2509_01416_amd import inputs as I


def _inst_1d(n, lx, st, ss, bc=(0, 0)):
    return I.Instance(nx=n, ny=1, lx=lx, ly=1.0, sigma_t=np.asarray(st, float).reshape(1, n),
                      sigma_s=np.asarray(ss, float).reshape(1, n),
                      source=np.zeros((1, n)), bc=tuple(bc) + (0, 0), dim=1)


def _dense_k(inst, quad, nsf):
    """Dominant eigenvalue and eigenvector of G diag(nu_sigma_f), with G
    assembled column by column from direct fixed-source solves."""
    n = inst.cells
    G = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        if inst.dim == 1:
            G[:, c] = solve_1d(inst.nx, inst.lx, quad.mu, quad.w, inst.sigma_t,
                               inst.sigma_s, e, bc=inst.bc[:2])
        else:
            G[:, c] = solve_2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta,
                               quad.w, inst.sigma_t, inst.sigma_s, e.reshape(inst.ny, inst.nx),
                               inst.bc).reshape(-1)
    A = G @ np.diag(np.asarray(nsf, float).reshape(-1))
    vals, vecs = np.linalg.eig(A)
    j = int(np.argmax(vals.real))
    v = np.real(vecs[:, j])
    v = v / E.fission_production(nsf.reshape(-1), v, E.cell_volume(inst))
    return float(vals[j].real), v


def test_infinite_medium_1d():
    n = 20
    inst = _inst_1d(n, 4.0, np.full(n, 1.0), np.full(n, 0.5), bc=(1, 1))
    nsf = np.full((1, n), 0.9)
    r = E.solve_eigen(inst, I.gauss_legendre(8), nsf)
    assert r.converged
    assert abs(r.k - 0.9 / 0.5) < 1e-9
    assert np.ptp(r.phi) < 1e-9 * np.max(r.phi)
    assert abs(E.fission_production(nsf, r.phi, E.cell_volume(inst)) - 1.0) < 1e-12


def test_infinite_medium_2d():
    inst = I.Instance(nx=6, ny=5, lx=3.0, ly=2.5, sigma_t=np.full((5, 6), 2.0),
                      sigma_s=np.full((5, 6), 1.2), source=np.zeros((5, 6)), bc=(1, 1, 1, 1))
    nsf = np.full((5, 6), 0.5)
    r = E.solve_eigen(inst, I.level_symmetric_2d(4), nsf)
    assert r.converged
    assert abs(r.k - 0.5 / 0.8) < 1e-9
    assert np.ptp(r.phi) < 1e-9 * np.max(r.phi)


@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_dense_eigensolve_1d(bc):
    rng = np.random.Generator(np.random.PCG64(3))
    n = 14
    st = rng.uniform(0.6, 1.8, n)
    ss = st * rng.uniform(0.2, 0.7, n)
    nsf = (st - ss) * rng.uniform(0.8, 2.5, n)
    nsf[3:6] = 0.0                                   # a non-fissile zone
    inst = _inst_1d(n, 5.0, st, ss, bc=bc)
    quad = I.gauss_legendre(8)
    k_ref, v_ref = _dense_k(inst, quad, nsf.reshape(1, n))
    r = E.solve_eigen(inst, quad, nsf.reshape(1, n), tol_k=1e-13, tol_phi=1e-12)
    assert r.converged
    assert abs(r.k - k_ref) < 1e-10 * k_ref, (r.k, k_ref)
    assert np.max(np.abs(r.phi.reshape(-1) - v_ref)) < 1e-8 * np.max(np.abs(v_ref))


def test_dense_eigensolve_2d():
    rng = np.random.Generator(np.random.PCG64(5))
    nx, ny = 5, 4
    st = rng.uniform(0.5, 1.5, (ny, nx))
    ss = st * rng.uniform(0.3, 0.8, (ny, nx))
    nsf = (st - ss) * rng.uniform(1.0, 2.0, (ny, nx))
    inst = I.Instance(nx=nx, ny=ny, lx=2.0, ly=1.5, sigma_t=st, sigma_s=ss,
                      source=np.zeros((ny, nx)), bc=(1, 0, 0, 1))
    quad = I.level_symmetric_2d(4)
    k_ref, v_ref = _dense_k(inst, quad, nsf)
    r = E.solve_eigen(inst, quad, nsf, tol_k=1e-13, tol_phi=1e-12)
    assert r.converged
    assert abs(r.k - k_ref) < 1e-10 * k_ref, (r.k, k_ref)
    assert np.max(np.abs(r.phi.reshape(-1) - v_ref)) < 1e-8 * np.max(np.abs(v_ref))


def test_eigen_case1_printed_k():
    """Eigen Case 1 (section 5.2; Table 7 model-based k = 1.71402):
    sigma_t = 1, sigma_s = 0.5, sigma_f = 0.3 on the 10 cm slab of section
    5.1 (100 cells, S32).  The paper gives no nu and no boundary condition;
    nu = 3 and vacuum faces are the reading.  The converged DD value under
    it is 1.71467 (S8 to S64 and 100 to 1000 cells agree to 1e-4), 0.04 %
    above the printed number, which came from solvers stopped at 1e-4;
    the pin allows 5e-4 relative."""
    n = 100
    inst = _inst_1d(n, 10.0, np.ones(n), np.full(n, 0.5))
    nsf = np.full((1, n), 3.0 * 0.3)
    r = E.solve_eigen(inst, I.gauss_legendre(32), nsf, tol_inner=1e-11,
                      tol_k=1e-10, tol_phi=1e-9)
    assert r.converged
    assert abs(r.k - 1.71402) / 1.71402 < 5e-4, r.k
    assert abs(r.k - 1.714665) < 2e-5, r.k
    # symmetric slab: symmetric eigenfunction, peaked at the centre
    phi = r.phi.reshape(-1)
    assert np.max(np.abs(phi - phi[::-1])) < 1e-8 * phi.max()
    assert np.argmax(phi) in (49, 50)


def test_linearity_and_start_independence():
    rng = np.random.Generator(np.random.PCG64(9))
    n = 30
    st = rng.uniform(0.8, 1.2, n)
    ss = 0.6 * st
    nsf = 0.5 * st
    inst = _inst_1d(n, 6.0, st, ss)
    quad = I.gauss_legendre(8)
    a = E.solve_eigen(inst, quad, nsf.reshape(1, n), tol_k=1e-12, tol_phi=1e-11)
    b = E.solve_eigen(inst, quad, 2.5 * nsf.reshape(1, n), tol_k=1e-12, tol_phi=1e-11)
    c = E.solve_eigen(inst, quad, nsf.reshape(1, n), tol_k=1e-12, tol_phi=1e-11,
                      phi0=rng.uniform(0.1, 1.0, (1, n)), k0=3.0)
    assert abs(b.k - 2.5 * a.k) < 1e-9 * b.k
    assert abs(c.k - a.k) < 1e-9 * a.k
    assert np.max(np.abs(c.phi - a.phi)) < 1e-8 * np.max(a.phi)
    # F(phi) = 1 after every update
    for r in (a, c):
        assert abs(E.fission_production(nsf, r.phi.reshape(-1), 6.0 / n) - 1.0) < 1e-12


# ------------------------------------------- neural-operator variants (A2) --

def _exact_linv_star(inst, quad, st_star, ss_star):
    """The exact inverse transport operator at uniform p* on the instance's
    grid (direct solve of the DD system)."""
    st = np.full((inst.ny, inst.nx), st_star)
    ss = np.full((inst.ny, inst.nx), ss_star)

    def linv(S):
        return solve_2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta, quad.w,
                        st, ss, S, inst.bc)
    return linv


@pytest.mark.parametrize("variant", ["sp", "cp"])
def test_no_variants_exact_when_only_scattering_changes(variant):
    """With sigma_t = sigma_t* the recast source (sigma_a* - sigma_a) phi is
    the exact change of the scattering term, so SP and CP driven by the
    exact operator at p* must converge to the model-based eigenpair."""
    rng = np.random.Generator(np.random.PCG64(13))
    nx, ny = 8, 7
    st_star, ss_star = 1.0, 0.8
    st = np.full((ny, nx), st_star)
    ss = rng.uniform(0.5, 0.9, (ny, nx))
    nsf = rng.uniform(0.2, 0.5, (ny, nx))
    inst = I.Instance(nx=nx, ny=ny, lx=4.0, ly=3.5, sigma_t=st, sigma_s=ss,
                      source=np.zeros((ny, nx)))
    quad = I.level_symmetric_2d(4)
    ref = E.solve_eigen(inst, quad, nsf, tol_k=1e-12, tol_phi=1e-11)
    r = E.solve_eigen_no(inst, quad, nsf, _exact_linv_star(inst, quad, st_star, ss_star),
                         st_star - ss_star, variant, tol_k=1e-12, tol_phi=1e-11)
    assert r.converged
    assert abs(r.k - ref.k) < 1e-9 * ref.k, (r.k, ref.k)
    assert np.max(np.abs(r.phi - ref.phi)) < 1e-8 * np.max(ref.phi)


def test_sp_linear_network_closed_form():
    """A pointwise network NO(S) = g S / sigma_a* on a uniform medium keeps
    every flux shape, and SP's fixed point solves
    g (nu_sigma_f / k + sigma_a* - sigma_a) / sigma_a* = 1."""
    from oracle import recast as RC
    n = 6
    g, sa_star, sa, nsf0 = 0.6, 0.2, 0.35, 0.3
    inst = I.Instance(nx=n, ny=n, lx=3.0, ly=3.0, sigma_t=np.full((n, n), 1.0),
                      sigma_s=np.full((n, n), 1.0 - sa), source=np.zeros((n, n)))
    linv = RC.network_inner(lambda x: g * x, sa_star)
    r = E.solve_eigen_no(inst, I.level_symmetric_2d(4), np.full((n, n), nsf0), linv, sa_star,
                         "sp", tol_k=1e-13, tol_phi=1e-12)
    assert r.converged
    exact = nsf0 / (sa_star / g - sa_star + sa)
    assert abs(r.k - exact) < 1e-11 * exact, (r.k, exact)


# ------------------------------------------------ three groups (section 5.3) --
# Tables 8-9: sigma_s^{g->h} (rows g, columns h), nu, sigma_t, sigma_f, chi.
MG_SS = [[0.024, 0.171, 0.033], [0.0, 0.600, 0.275], [0.0, 0.0, 2.000]]
MG_NU = [3.0, 2.5, 2.0]
MG_ST = [0.240, 0.975, 3.000]
MG_SF = [0.006, 0.060, 0.900]
MG_CHI = [0.96, 0.04, 0.0]


def _mg_fields(shape, ss=MG_SS, st=MG_ST, nsf=None):
    G = len(st)
    nsf = [MG_NU[g] * MG_SF[g] for g in range(G)] if nsf is None else nsf
    sigma_s = [[np.full(shape, ss[g][h]) if (h >= g and ss[g][h] != 0.0) else None
                for h in range(G)] for g in range(G)]
    return ([np.full(shape, st[g]) for g in range(G)], sigma_s,
            [np.full(shape, nsf[g]) for g in range(G)])


def test_three_group_printed_k():
    """Table 10 model-based k = 1.30621 on the section 5.1 slab (10 cm,
    100 cells, S32; vacuum faces as for eigen Case 1)."""
    n = 100
    inst = _inst_1d(n, 10.0, np.ones(n), np.zeros(n))
    st, ss, nsf = _mg_fields((1, n))
    r = E.solve_eigen_mg(inst, I.gauss_legendre(32), st, ss, nsf, MG_CHI, tol_inner=1e-11,
                         tol_k=1e-11, tol_phi=1e-10)
    assert r.converged
    assert abs(r.k - 1.30621) < 1e-5 * 1.30621, r.k
    # the fast group peaks where fissions are, the thermal flux tracks it
    assert np.all(r.phi > 0)


def test_three_group_infinite_medium():
    """Reflective on every face with uniform data: k_inf is the dominant
    eigenvalue of the 3 x 3 balance nu_sigma_f^T A^-1 chi with
    A = diag(sigma_t) - S^T (S[g][h] = sigma_s^{g->h}); 1.72 for Tables 8-9."""
    A = np.diag(MG_ST) - np.array(MG_SS).T
    nsf = np.array(MG_NU) * np.array(MG_SF)
    k_inf = float(nsf @ np.linalg.solve(A, np.array(MG_CHI)))
    assert abs(k_inf - 1.72) < 1e-12
    inst = I.Instance(nx=5, ny=4, lx=2.0, ly=2.0, sigma_t=np.ones((4, 5)),
                      sigma_s=np.zeros((4, 5)), source=np.zeros((4, 5)), bc=(1, 1, 1, 1))
    st, ss, nsf_f = _mg_fields((4, 5))
    r = E.solve_eigen_mg(inst, I.level_symmetric_2d(4), st, ss, nsf_f, MG_CHI)
    assert r.converged
    assert abs(r.k - k_inf) < 1e-9 * k_inf
    spec = np.linalg.solve(A, np.array(MG_CHI))            # group flux ratios
    got = np.array([p.mean() for p in r.phi])
    assert np.allclose(got / got.sum(), spec / spec.sum(), rtol=1e-9)


def test_three_group_dense_eigensolve():
    """k and the group fluxes from the dominant eigenpair of the map
    fission density -> new fission density, assembled column by column with
    direct DD solves per group (downscatter applied in group order)."""
    rng = np.random.Generator(np.random.PCG64(17))
    n = 10
    inst = _inst_1d(n, 4.0, np.ones(n), np.zeros(n), bc=(1, 0))
    st = [rng.uniform(0.2, 0.4, n), rng.uniform(0.8, 1.2, n), rng.uniform(2.0, 3.5, n)]
    ss_full = [[st[0] * 0.1, st[0] * 0.6, st[0] * 0.1],
               [None, st[1] * 0.6, st[1] * 0.3],
               [None, None, st[2] * 0.6]]
    nsf = [st[0] * 0.05, st[1] * 0.1, st[2] * 0.5]
    nsf[2][2:4] = 0.0
    chi = [0.9, 0.1, 0.0]
    quad = I.gauss_legendre(8)

    def groups_from_fission(fd):
        ph = []
        for g in range(3):
            q = chi[g] * fd
            for h in range(g):
                if ss_full[h][g] is not None:
                    q = q + ss_full[h][g] * ph[h]
            ph.append(solve_1d(n, 4.0, quad.mu, quad.w, st[g], ss_full[g][g], q, bc=(1, 0)))
        return ph
    Mx = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        Mx[:, c] = sum(f * p for f, p in zip(nsf, groups_from_fission(e)))
    vals, vecs = np.linalg.eig(Mx)
    j = int(np.argmax(vals.real))
    k_ref = float(vals[j].real)
    fd = np.real(vecs[:, j])
    ph = np.array(groups_from_fission(fd))
    ph = ph / E.fission_production_mg(nsf, ph, 0.4)
    r = E.solve_eigen_mg(inst, quad, [a.reshape(1, n) for a in st],
                         [[None if a is None else a.reshape(1, n) for a in row] for row in ss_full],
                         [a.reshape(1, n) for a in nsf], chi, tol_k=1e-13, tol_phi=1e-12)
    assert r.converged
    assert abs(r.k - k_ref) < 1e-10 * k_ref, (r.k, k_ref)
    assert np.max(np.abs(r.phi.reshape(3, n) - ph)) < 1e-8 * np.max(np.abs(ph))
