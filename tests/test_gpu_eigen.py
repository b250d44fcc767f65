"""Parity of the HIP k-eigenvalue path (tr_eigen) against the FP64 oracle.

Section 5.2 Eq. 26 with the power iteration of Appendix A2 (Eq. A1-A4).
The device runs FP32 fields with FP64 sums.  Tolerances:
  * the device stops at |dk|/k < 1e-6 and max|dphi|/max|phi| < 1e-5 with
    inner solves to a relative L2 change of 1e-6; the oracle runs to
    1e-10 / 1e-12.  Near the limit the outer error contracts by the
    dominance ratio d per update, so what is left after the stop is about
    d / (1 - d) times the last change; the inner solves add an error of
    the order of their tolerance times the inverse spectral gap of the
    scattering iteration (<= 10 here).  With d / (1 - d) <= 10 for these
    problems the bars are: k within 1e-5 relative, the normalised
    eigenfunction within 2e-4 relative (max norm).  The FP64 oracle under
    the same stopping rules lands within 2e-6 (k) and 7.5e-5 (phi) of its
    tight solution on these cases; FP32 rounding adds about 1e-6.
"""
import numpy as np
import pytest

from gpu_util import log, rel_inf, to_problem
from oracle import eigen as E
from paper_2509_01416_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = dict(tol_k=1e-6, tol_phi=1e-5, tol_inner=1e-6, max_outer=300, max_inner=5000)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01416_amd import binding as B
    assert torch.cuda.is_available()
    ctx = B.Context()
    yield torch, B, ctx
    ctx.close()


def _dev(torch, a, inst):
    shape = (inst.nx,) if inst.dim == 1 else (inst.ny, inst.nx)
    return torch.tensor(np.asarray(a, np.float32).reshape(shape), device="cuda")


def _run(env, insts, quad, nsfs, phi0=None, k0=None, **kw):
    torch, B, ctx = env
    probs = [to_problem(i, torch) for i in insts]
    nsf = [_dev(torch, f, i) for f, i in zip(nsfs, insts)]
    phis = [torch.zeros_like(p.sigma_t) for p in probs]
    init = None if phi0 is None else [_dev(torch, p, i) for p, i in zip(phi0, insts)]
    args = dict(TOL)
    args.update(kw)
    rc, st = B.tr_eigen(ctx, probs, nsf, B.Quad.from_inputs(quad), init, phis, k0, **args)
    torch.cuda.synchronize()
    return rc, st, [p.cpu().numpy().astype(np.float64).reshape(i.ny, i.nx)
                    for p, i in zip(phis, insts)]


def _slab(n, lx, st, ss, bc=(0, 0)):
    return I.Instance(nx=n, ny=1, lx=lx, ly=1.0, sigma_t=np.asarray(st, float).reshape(1, n),
                      sigma_s=np.asarray(ss, float).reshape(1, n),
                      source=np.zeros((1, n)), bc=tuple(bc) + (0, 0), dim=1)


def _hetero(nx, ny, seed, bc=(0, 0, 0, 0), lx=6.0, ly=6.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    st = rng.uniform(0.6, 1.6, (ny, nx))
    ss = st * rng.uniform(0.3, 0.7, (ny, nx))
    nsf = (st - ss) * rng.uniform(1.2, 2.4, (ny, nx))
    inst = I.Instance(nx=nx, ny=ny, lx=lx, ly=ly, sigma_t=st, sigma_s=ss,
                      source=np.zeros((ny, nx)), bc=bc)
    return inst, nsf


def test_eigen_case1_slab(env):
    """Eigen Case 1 (Table 7, k = 1.71402) under the reading nu = 3 and
    vacuum faces: 100 cells on 10 cm, S32."""
    B = env[1]
    n = 100
    inst = _slab(n, 10.0, np.ones(n), np.full(n, 0.5))
    nsf = np.full((1, n), 0.9)
    quad = I.gauss_legendre(32)
    log("eigen case 1: 1-D slab 100 cells S32")
    rc, st, phi = _run(env, [inst], quad, [nsf])
    ref = E.solve_eigen(inst, quad, nsf, tol_inner=1e-12, tol_k=1e-11, tol_phi=1e-10)
    log(f"  k gpu={st[0]['k']:.7f} oracle={ref.k:.7f} outer={st[0]['outer']} "
        f"inner={st[0]['inner']} balance={st[0]['balance_rel']:.1e}")
    assert rc == B.TR_OK and st[0]["status"] == B.TR_OK
    assert abs(st[0]["k"] - ref.k) < 1e-5 * ref.k
    assert abs(st[0]["k"] - 1.71402) < 5e-4 * 1.71402
    assert rel_inf(phi[0], ref.phi) < 2e-4
    assert abs(E.fission_production(nsf, phi[0], 0.1) - 1.0) < 1e-5
    assert st[0]["balance_rel"] < 1e-4


def test_eigen_batch_2d_specialised(env):
    """A batch of heterogeneous vacuum problems whose launch plan takes the
    specialised sweep (vacuum faces, 64-row segments), S8."""
    torch, B, ctx = env
    cases = [_hetero(128, 128, 21), _hetero(128, 64, 22, lx=8.0, ly=4.0)]
    insts = [c[0] for c in cases]
    nsfs = [c[1] for c in cases]
    quad = I.level_symmetric_2d(8)
    probs = [to_problem(i, torch) for i in insts]
    assert ctx.sweep_plan(probs, B.Quad.from_inputs(quad))["specialised"] == 1
    log("eigen 2-D batch (specialised sweep): 128x128 + 128x64 S8")
    rc, st, phi = _run(env, insts, quad, nsfs)
    assert rc == B.TR_OK
    for j, (inst, nsf) in enumerate(cases):
        ref = E.solve_eigen(inst, quad, nsf, tol_inner=1e-12, tol_k=1e-10, tol_phi=1e-10)
        log(f"  [{j}] k gpu={st[j]['k']:.7f} oracle={ref.k:.7f} outer={st[j]['outer']} "
            f"inner={st[j]['inner']} balance={st[j]['balance_rel']:.1e}")
        assert st[j]["status"] == B.TR_OK
        assert abs(st[j]["k"] - ref.k) < 1e-5 * ref.k
        assert rel_inf(phi[j], ref.phi) < 2e-4
        assert st[j]["balance_rel"] < 1e-4


def test_eigen_batch_2d_generic_reflective(env):
    """Mixed sizes with reflective faces (the generic sweep): each instance
    stops on its own test; an infinite medium gives nu_sigma_f / sigma_a."""
    torch, B, ctx = env
    a = _hetero(24, 16, 31, bc=(1, 0, 0, 1), lx=3.0, ly=2.0)
    b = _hetero(40, 33, 32, bc=(0, 0, 1, 0), lx=5.0, ly=4.0)
    inf = I.Instance(nx=20, ny=12, lx=2.0, ly=1.2, sigma_t=np.full((12, 20), 1.5),
                     sigma_s=np.full((12, 20), 0.9), source=np.zeros((12, 20)),
                     bc=(1, 1, 1, 1))
    nsf_inf = np.full((12, 20), 0.75)
    insts = [a[0], b[0], inf]
    nsfs = [a[1], b[1], nsf_inf]
    quad = I.level_symmetric_2d(8)
    log("eigen 2-D batch (generic sweep): 24x16 refl, 40x33 refl, 20x12 infinite medium")
    rc, st, phi = _run(env, insts, quad, nsfs)
    assert rc == B.TR_OK
    for j, (inst, nsf) in enumerate(zip(insts, nsfs)):
        ref = E.solve_eigen(inst, quad, nsf, tol_inner=1e-12, tol_k=1e-10, tol_phi=1e-10)
        log(f"  [{j}] k gpu={st[j]['k']:.7f} oracle={ref.k:.7f} outer={st[j]['outer']}")
        assert st[j]["status"] == B.TR_OK
        assert abs(st[j]["k"] - ref.k) < 1e-5 * ref.k
        assert rel_inf(phi[j], ref.phi) < 2e-4
    assert abs(st[2]["k"] - 0.75 / 0.6) < 1e-5 * 1.25
    outers = {s["outer"] for s in st}
    assert len(outers) > 1          # the instances finished at different updates


def test_eigen_warm_start_and_repeatability(env):
    """Started from a converged pair the loop stops after one or two
    updates with the same k; two identical calls agree bit for bit."""
    B = env[1]
    inst, nsf = _hetero(48, 48, 41)
    quad = I.level_symmetric_2d(8)
    rc1, st1, phi1 = _run(env, [inst], quad, [nsf])
    rc2, st2, phi2 = _run(env, [inst], quad, [nsf])
    assert rc1 == rc2 == B.TR_OK
    assert st1[0]["k"] == st2[0]["k"] and np.array_equal(phi1[0], phi2[0])
    rc3, st3, phi3 = _run(env, [inst], quad, [nsf], phi0=[phi1[0]], k0=[st1[0]["k"]])
    log(f"  cold outer={st1[0]['outer']} warm outer={st3[0]['outer']}")
    assert rc3 == B.TR_OK and st3[0]["outer"] <= 2
    assert abs(st3[0]["k"] - st1[0]["k"]) < 3e-6 * st1[0]["k"]
    assert rel_inf(phi3[0], phi1[0]) < 3e-5


def test_eigen_not_converged_and_invalid(env):
    torch, B, ctx = env
    inst, nsf = _hetero(32, 32, 51)
    quad = I.level_symmetric_2d(4)
    rc, st, _ = _run(env, [inst], quad, [nsf], max_outer=2)
    assert rc == B.TR_NOT_CONVERGED and st[0]["outer"] == 2
    for bad in (np.zeros_like(nsf), -nsf):
        probs = [to_problem(inst, torch)]
        phi = [torch.zeros_like(probs[0].sigma_t)]
        rc, _ = B.tr_eigen(ctx, probs, [_dev(torch, bad, inst)], B.Quad.from_inputs(quad),
                           None, phi, None, raise_on_error=False, **TOL)
        assert rc == B.TR_ERR_INVALID_ARG
    rc, _ = B.tr_eigen(ctx, [to_problem(inst, torch)], [_dev(torch, nsf, inst)],
                       B.Quad.from_inputs(quad), None, phi, [0.0], raise_on_error=False, **TOL)
    assert rc == B.TR_ERR_INVALID_ARG
