"""tr_solve_noalloc (every workspace in the library's fixed device scratch)
against tr_solve, through the C ABI: two calls in a row, the second with a
smaller input, each bit for bit equal to tr_solve on the same problems (the
same kernels and launch shapes), and a problem set too large for the
scratch rejected before any launch."""
import numpy as np
import pytest

from gpu_util import log, to_problem
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


def _both(env, insts, quad, tol, max_iter):
    torch, B, ctx = env
    probs = [to_problem(i, torch) for i in insts]
    q = B.Quad.from_inputs(quad)
    out = []
    for noalloc in (False, True):
        phis = [torch.full_like(p.sigma_t, 7.0) for p in probs]   # stale values
        rc, st = B.tr_solve(ctx, probs, q, None, phis, tol, max_iter, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append((rc, st, [p.cpu().numpy() for p in phis]))
    return out


def _same(ref, got):
    (rc0, st0, p0), (rc1, st1, p1) = ref, got
    assert rc0 == rc1 == 0
    for a, b in zip(st0, st1):
        assert a["iterations"] == b["iterations"] and a["residual"] == b["residual"]
        assert a["balance_rel"] == b["balance_rel"]
    for a, b in zip(p0, p1):
        assert np.array_equal(a, b)


def test_noalloc_matches_tr_solve_two_calls(env):
    torch, B, ctx = env
    # call 1: the 16 x 256^2 S16 benchmark batch under the error-bound rule
    # (snapshots in the scratch too), near the scratch's size
    wl = I.hard_two_region(16, 256)
    log("[tr_solve_noalloc] 16 x 256^2 S16, error-bound rule")
    ctx.set_stop_rule("bound")
    try:
        r = _both(env, wl.instances, wl.quad, 1e-6, 3000)
    finally:
        ctx.set_stop_rule("change")
    log(f"  iterations {[s['iterations'] for s in r[1][1]]}")
    _same(*r)
    # call 2: smaller, uneven, with reflective faces (the generic sweep)
    log("[tr_solve_noalloc] three small problems, reflective faces")
    insts = [I.random_instance(96, 80, seed=1, bc=(1, 0, 1, 0)),
             I.random_instance(64, 64, seed=2, bc=(0, 1, 0, 0)),
             I.random_instance(40, 56, seed=3)]
    r = _both(env, insts, I.level_symmetric_2d(8), 1e-7, 5000)
    log(f"  iterations {[s['iterations'] for s in r[1][1]]}")
    _same(*r)


def test_noalloc_rejects_a_workspace_beyond_the_scratch(env):
    """64 problems of 256 x 256 at S16 need about 350 MB of workspace: an
    argument error with a message, nothing launched, and the next call on
    the same context works."""
    torch, B, ctx = env
    inst = I.hard_two_region(1, 256).instances[0]
    p = to_problem(inst, torch)
    q = B.Quad.from_inputs(I.level_symmetric_2d(16))
    phis = [torch.zeros_like(p.sigma_t) for _ in range(64)]
    rc, _ = B.tr_solve(ctx, [p] * 64, q, None, phis, 1e-6, 10, raise_on_error=False,
                       noalloc=True)
    msg = ctx.last_error()
    log(f"  64 x 256^2: status {rc}: {msg}")
    assert rc == B.TR_ERR_INVALID_ARG and "fixed scratch" in msg
    assert all(float(f.abs().max()) == 0.0 for f in phis)
    small = I.random_instance(32, 32, seed=9)
    r = _both(env, [small], I.level_symmetric_2d(4), 1e-7, 2000)
    _same(*r)
