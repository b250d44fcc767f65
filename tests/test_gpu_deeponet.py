"""The DeepONet (section 4.1, Eq. 11) on the matrix cores against the FP64
oracle, through the C ABI, and as the operator of the recast loop (Eq. 24).

The ReLU masks are decisions: a pre-activation within rounding of zero can
fall on different sides in FP32 and FP64.  The gradient tests therefore
shift each bias until every pre-activation of the test inputs lies at least
1e-5 of its layer's scale away from zero, so that both sides take the same
decisions (the trunk's smooth coordinate input otherwise puts hundreds of
its 819,200 pre-activations near zero).

Bars as for the Fourier operator (tests/test_gpu_fno.py): FP32 operands
1e-5 relative L2 on outputs and gradients; BF16 operands 1e-2 with
gradient cosine > 0.999.  The trunk's first-layer gradients (V1, c1) are
sums over the 4096 cells of terms of both signs that cancel to about a
thousandth of their magnitude; their error is measured relative to the sum
of the magnitudes of the terms (the scale of FP32 rounding in any sum) at
the same bars."""
import numpy as np
import pytest

from gpu_util import log, rel_l2, to_problem
from oracle import deeponet as D
from oracle import recast as RC
from paper_2509_01416_amd import inputs as I

pytestmark = pytest.mark.gpu

LAY = D.Layout()
N = 64


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01416_amd import binding as B
    assert torch.cuda.is_available()
    ctx = B.Context()
    yield torch, B, ctx
    ctx.close()


def _params(seed):
    return D.init_params(LAY, seed).astype(np.float32)


def _fields(batch, seed):
    return np.stack([I.grf_2d(N, 10.0, seed=seed + b, mean=1.0, std=0.3)
                     for b in range(batch)])


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _oracle(p, x):
    return D.forward(p.astype(np.float64), x.reshape(x.shape[0], -1), D.grid_coords(N), LAY)


def _margined(p, x, margin=1e-5):
    """Parameters whose biases are shifted so that no pre-activation of the
    inputs x lies within margin x (its layer's largest magnitude) of zero:
    each unit's zero is moved to the middle of the widest gap between the
    sorted pre-activation values near it."""
    q = D.unpack(p.astype(np.float64), LAY)
    u, y = x.reshape(x.shape[0], -1).astype(np.float64), D.grid_coords(N)
    for (W, b), inp in ((("W1", "b1"), "u"), (("W2", "b2"), "a1"),
                        (("V1", "c1"), "y"), (("V2", "c2"), "g1")):
        _, cache = D.forward(D.pack(q, LAY), u, y, LAY)
        src = {"u": u, "y": y, "a1": cache["a1"], "g1": cache["g1"]}[inp]
        z = src @ q[W] + q[b]
        scale = np.abs(z).max()
        for j in range(z.shape[1]):
            v = np.sort(z[:, j])
            if v[0] > margin * scale or v[-1] < -margin * scale:
                continue
            i0 = int(np.searchsorted(v, 0.0))
            lo, hi = max(1, i0 - 40), min(len(v) - 1, i0 + 40)
            i = lo + int(np.argmax(v[lo:hi + 1] - v[lo - 1:hi]))
            q[b][j] -= 0.5 * (v[i - 1] + v[i])
        z = src @ q[W] + q[b]
        assert np.abs(z).min() > margin * scale, (W, np.abs(z).min() / scale)
    return D.pack(q, LAY).astype(np.float32)


def test_param_count_and_roundtrip(env):
    torch, B, ctx = env
    p = _params(1)
    m = B.Model(ctx, p, arch="deeponet")
    assert m.n_params == 940_600 == LAY.count()
    assert np.array_equal(m.get_params(), p)
    m.close()


@pytest.mark.parametrize("fp32,tol", [(True, 1e-5), (False, 1e-2)])
def test_forward_parity(env, fp32, tol):
    """Batches of 3 and 300 (the branch's first contraction is split over K
    below 257 samples and not above)."""
    torch, B, ctx = env
    p = _params(3)
    m = B.Model(ctx, p, arch="deeponet")
    m.set_fp32(fp32)
    for batch in (3, 300):
        x = _fields(3, 700)
        x = np.concatenate([x] * (batch // 3))
        out = m.forward(_dev(torch, x)).cpu().numpy().reshape(batch, -1)
        ref, _ = _oracle(p, x)
        e = rel_l2(out, ref)
        log(f"  forward fp32={fp32} batch {batch}: rel_l2={e:.3e} (bar {tol})")
        assert e < tol
    m.close()


@pytest.mark.parametrize("fp32", [True, False])
def test_gradient_parity(env, fp32):
    torch, B, ctx = env
    x = _fields(5, 800)
    t = _fields(5, 900) * 0.1
    p = _margined(_params(4), x)
    m = B.Model(ctx, p, arch="deeponet")
    m.set_fp32(fp32)
    g = torch.zeros(m.n_params, dtype=torch.float32, device="cuda")
    loss = m.train_step(_dev(torch, x), _dev(torch, t), 0.0, grad_out=g)
    g = g.cpu().numpy().astype(np.float64)
    out, cache = _oracle(p, x)
    d = out - t.reshape(5, -1)
    ref_loss = float(np.mean(d * d))
    parts = {}
    gref = D.backward(p.astype(np.float64), cache, 2.0 * d / d.size, LAY, parts)
    # magnitudes of the terms of the trunk's first-layer sums
    mag = {"V1": (np.abs(cache["y"]).T @ np.abs(parts["gt1"])).reshape(-1),
           "c1": np.abs(parts["gt1"]).sum(axis=0)}
    le = abs(loss - ref_loss) / ref_loss
    log(f"  loss fp32={fp32}: {loss:.6e} vs {ref_loss:.6e} (rel {le:.2e})")
    assert le < (1e-5 if fp32 else 1e-2)
    o = 0
    for name, sh in LAY.shapes():
        n = int(np.prod(sh))
        a, b = g[o:o + n], gref[o:o + n]
        o += n
        e = rel_l2(a, b)
        if name in mag:
            e = float(np.linalg.norm(a - b) / np.linalg.norm(mag[name]))
            cancel = float(np.linalg.norm(b) / np.linalg.norm(mag[name]))
            log(f"  grad {name}: error / |terms| = {e:.2e} (sum / |terms| = {cancel:.1e})")
            assert e < (1e-5 if fp32 else 1e-2), name
            continue
        if fp32:
            log(f"  grad {name}: rel_l2={e:.2e}")
            assert e < 1e-5, name
        else:
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
            log(f"  grad {name}: rel_l2={e:.2e} cosine={cos:.6f}")
            assert e < 3e-2 and cos > 0.999, name
    assert np.array_equal(m.get_params(), p)
    m.close()


def test_training_reduces_loss_and_refreshes_the_basis(env):
    """Adam steps lower the loss; the forward after training uses the new
    trunk basis (it matches a fresh model built from the trained
    parameters bit for bit)."""
    torch, B, ctx = env
    x = _fields(8, 1200)
    t = 0.5 * x + 0.2
    m = B.Model(ctx, _params(6), arch="deeponet")
    xd, td = _dev(torch, x), _dev(torch, t)
    m.forward(xd)
    losses = [m.train_step(xd, td, 1e-4) for _ in range(30)]
    log(f"  training: loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    a = m.forward(xd).cpu().numpy()
    fresh = B.Model(ctx, m.get_params(), arch="deeponet")
    b = fresh.forward(xd).cpu().numpy()
    assert np.array_equal(a, b)
    m.close()
    fresh.close()


def test_recast_parity_with_oracle(env):
    """Five recast updates (tol 0) with a DeepONet in FP32 mode against the
    oracle loop driving the FP64 DeepONet."""
    torch, B, ctx = env
    p = _params(8)
    m = B.Model(ctx, p, arch="deeponet")
    m.set_fp32(True)
    wl = I.fno_eval_set("line", count=2)
    probs = [to_problem(i, torch) for i in wl.instances]
    outs = [torch.zeros_like(pr.sigma_t) for pr in probs]
    rc, st = B.no_recast_guess(ctx, m, probs, I.SIGMA_T_STAR, I.SIGMA_S_STAR, 0.0, 5, outs)
    sa_star = I.SIGMA_T_STAR - I.SIGMA_S_STAR

    def net(s):
        out, _ = _oracle(p, s[None])
        return out[0].reshape(N, N)
    inner = RC.network_inner(net, sa_star)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    for inst, o, s in zip(wl.instances, outs, st):
        phi, ost, it, _ = RC.recast_loop(f32(inst.source), f32(inst.sigma_t) - f32(inst.sigma_s),
                                         sa_star, inner, tol=0.0, max_iter=5)
        e = rel_l2(o.cpu().numpy(), phi)
        log(f"  recast: iters={s['iterations']} rel_l2={e:.2e}")
        assert s["iterations"] == it == 5 and e < 1e-5
    m.close()


def test_bad_shape_rejected(env):
    torch, B, ctx = env
    rc = ctx.lib.no_model_create_deeponet(ctx.handle, None, 64, 200, 100, None)
    assert rc == B.TR_ERR_INVALID_ARG
    import ctypes
    h = ctypes.c_void_p()
    rc = ctx.lib.no_model_create_deeponet(ctx.handle, ctypes.byref(h), 32, 200, 100, None)
    assert rc == B.TR_ERR_INVALID_ARG and "unsupported DeepONet" in ctx.last_error()
