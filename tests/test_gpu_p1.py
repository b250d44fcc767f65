"""Linearly anisotropic (P1) scattering (section 5.1 Eq. 25) on the GPU,
against the oracle, through the C ABI.

Bars as for the isotropic solves (tests/test_gpu_si.py): 1e-5 relative L2
against the oracle's fixed point.  The paper's Cases 2 and 3 are 1-D slabs
(S32, 100 cells); the x-y problems run the generic sweep with the current
planes.  The network warm start (Case 2 analogue on the network grid) shows
the model-based iteration correcting a guess that cannot see the P1 term
(Eq. 23's isotropic reading)."""
import numpy as np
import pytest

import oracle
from gpu_util import log, rel_l2, to_problem
from paper_2509_01416_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01416_amd import binding as B
    assert torch.cuda.is_available()
    ctx = B.Context()
    yield torch, B, ctx
    ctx.close()


def _solve(env, insts, quad, tol, phi0=None, max_iter=20000):
    torch, B, ctx = env
    probs = [to_problem(i, torch) for i in insts]
    out = [torch.zeros_like(p.sigma_t) for p in probs]
    rc, st = B.tr_solve(ctx, probs, B.Quad.from_inputs(quad), phi0, out, tol, max_iter)
    torch.cuda.synchronize()
    return rc, st, [o.cpu().numpy().astype(np.float64).reshape(i.ny, i.nx)
                    for o, i in zip(out, insts)]


@pytest.mark.parametrize("case", [2, 3])
def test_paper_slab_cases_p1(env, case):
    """The paper's Case 2 and Case 3 slabs (P1, sigma_s1 = 0.3): GPU solve
    (max-relative change 1e-9) against the oracle's fixed point; the P1
    term moves the answer well beyond the bar."""
    wl = I.paper_slab_p1(case)
    inst = wl.instances[0]
    rc, st, phis = _solve(env, [inst], wl.quad, -1e-9)
    ref = oracle.solve_instance(inst, wl.quad, tol=1e-14, f32_inputs=True)
    iso = oracle.solve_instance(I.Instance(**{**inst.__dict__, "sigma_s1": None}), wl.quad,
                                tol=1e-14, f32_inputs=True)
    e = rel_l2(phis[0], ref.phi.reshape(1, -1))
    d = rel_l2(iso.phi, ref.phi)
    log(f"  case {case}: iterations {st[0]['iterations']} (oracle {ref.iterations}), "
        f"rel_l2 {e:.2e}, balance {st[0]['balance_rel']:.1e}; P1 effect {d:.2e}")
    assert rc == 0 and e < 1e-5 and st[0]["balance_rel"] < 1e-4
    assert d > 1e-3


def test_p1_two_dimensional_batch(env):
    """A batch of x-y problems with P1 scattering in one launch (64-row and
    32-row segments, reflective faces, one problem without sigma_s1):
    every answer against the oracle's fixed point; the isotropic problem's
    answer equals its solve in an isotropic batch to FP32 rounding."""
    quad = I.level_symmetric_2d(8)
    insts = [I.random_instance(64, 64, seed=71, c_range=(0.5, 0.9)),
             I.random_instance(48, 32, seed=72, c_range=(0.5, 0.9), bc=(1, 0, 1, 0)),
             I.random_instance(40, 64, seed=73, c_range=(0.5, 0.9)),
             I.random_instance(32, 32, seed=74, c_range=(0.5, 0.9))]
    for k, inst in enumerate(insts[:3]):
        rng = np.random.Generator(np.random.PCG64(80 + k))
        inst.sigma_s1 = inst.sigma_s * rng.uniform(-0.4, 0.6, inst.sigma_s.shape)
    torch, B, ctx = env
    plan = ctx.sweep_plan([to_problem(i, torch) for i in insts], B.Quad.from_inputs(quad))
    assert plan["D"] == 1 and plan["specialised"] == 0
    rc, st, phis = _solve(env, insts, quad, 1e-7)
    log(f"  status {rc}: iterations {[s['iterations'] for s in st]}, "
        f"residuals {[float('%.2g' % s['residual']) for s in st]}")
    assert rc == 0
    for inst, s, phi in zip(insts, st, phis):
        ref = oracle.solve_instance(inst, quad, tol=1e-13, f32_inputs=True)
        e = rel_l2(phi, ref.phi)
        log(f"  {inst.nx}x{inst.ny} bc={inst.bc} p1={inst.sigma_s1 is not None}: "
            f"iterations {s['iterations']} (oracle {ref.iterations}), rel_l2 {e:.2e}, "
            f"balance {s['balance_rel']:.1e}")
        assert e < 1e-5 and s["balance_rel"] < 1e-4
    _, _, alone = _solve(env, insts[3:], quad, 1e-7)
    assert rel_l2(phis[3], alone[0]) < 1e-6


def test_p1_recast_guess_corrected_by_the_iteration(env):
    """Case 2 analogue on the network grid: the recast guess (the network
    sees the isotropic problem only) sits closer to the isotropic solution
    than to the P1 one; source iteration from it converges to the P1
    oracle solution within the bar, in fewer sweeps than from zero."""
    torch, B, ctx = env
    from paper_2509_01416_amd import train as T
    model = B.Model(ctx, T.load_weights())
    wl = I.p1_eval_set(4)
    probs = [to_problem(i, torch) for i in wl.instances]
    quad = B.Quad.from_inputs(wl.quad)
    guess = [torch.zeros_like(p.sigma_t) for p in probs]
    B.no_recast_guess(ctx, model, probs, I.SIGMA_T_STAR, I.SIGMA_S_STAR, 1e-3, 30, guess)
    g = [x.cpu().numpy().astype(np.float64) for x in guess]
    warm = [x.clone() for x in guess]
    _, sw = B.tr_solve(ctx, probs, quad, warm, warm, 1e-7, 20000)
    zero = [torch.zeros_like(p.sigma_t) for p in probs]
    _, sz = B.tr_solve(ctx, probs, quad, None, zero, 1e-7, 20000)
    for k, inst in enumerate(wl.instances):
        ref = oracle.solve_instance(inst, wl.quad, tol=1e-13, f32_inputs=True)
        iso = oracle.solve_instance(I.Instance(**{**inst.__dict__, "sigma_s1": None}),
                                    wl.quad, tol=1e-13, f32_inputs=True)
        e = rel_l2(warm[k].cpu().numpy(), ref.phi)
        g_p1, g_iso = rel_l2(g[k], ref.phi), rel_l2(g[k], iso.phi)
        log(f"  instance {k}: guess vs P1 {g_p1:.2e}, vs isotropic {g_iso:.2e}; "
            f"sweeps warm {sw[k]['iterations']} zero {sz[k]['iterations']}; final {e:.2e}")
        assert e < 1e-5
        assert g_iso < g_p1
        assert sw[k]["iterations"] < sz[k]["iterations"]
    model.close()


def test_p1_rejections(env):
    """|sigma_s1| > sigma_s and non-finite values are argument errors; the
    eigenvalue solvers reject P1 problems; a bare sweep ignores sigma_s1."""
    torch, B, ctx = env
    quad = B.Quad.from_inputs(I.level_symmetric_2d(4))
    inst = I.random_instance(16, 16, seed=5)
    for bad, want in ((1.5 * inst.sigma_s, B.TR_ERR_INVALID_ARG),
                      (np.where(np.arange(256).reshape(16, 16) == 9, np.inf, 0.1 * inst.sigma_s),
                       B.TR_ERR_NONFINITE)):
        inst.sigma_s1 = bad
        p = to_problem(inst, torch)
        out = [torch.zeros_like(p.sigma_t)]
        rc, _ = B.tr_solve(ctx, [p], quad, None, out, 1e-6, 100, raise_on_error=False)
        assert rc == want, rc
    inst.sigma_s1 = 0.2 * inst.sigma_s
    p = to_problem(inst, torch)
    rc, _ = B.tr_eigen(ctx, [p], [torch.full_like(p.sigma_t, 0.1)], quad, None,
                       [torch.zeros_like(p.sigma_t)], raise_on_error=False)
    assert rc == B.TR_ERR_INVALID_ARG and "isotropic" in ctx.last_error()
    em = torch.ones_like(p.sigma_t)
    a, b = torch.zeros_like(em), torch.zeros_like(em)
    B.tr_sweep(ctx, [p], quad, [em], [a])
    p.sigma_s1 = None
    B.tr_sweep(ctx, [p], quad, [em], [b])
    assert torch.equal(a, b)
