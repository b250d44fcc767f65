"""Training of the 2-D operator network on solver-generated data
(arXiv 2509.01416 section 5.2 and Appendix A1, carried to 2-D).

The data are solutions of the transport problem at the single training
configuration p* = (sigma_t* = 1, sigma_s* = 0.8) on the 64 x 64 grid of a
10 x 10 mfp square with vacuum faces, one per seeded Gaussian-random-field
source, computed by the library's own batched source iteration (S8, relative
change 1e-7).  The network learns the scaled map
    S / s  ->  sigma_a* phi / s,     s = mean |S|,
which is exact to rescale because the transport solution is linear in S.
Training: MSE loss, Adam (0.9, 0.999, 1e-8) at a constant lr 1e-3, batch 32,
a 1800 / 200 train / validation split, FP32 master weights and BF16 operands
on the matrix cores; every forward and backward step runs in the library's
kernels (no_train_step).  The epoch budget is wall time; the parameters kept
are those of the best validation error (checked every 5 epochs), since the
constant learning rate leaves the error oscillating late in training.

A run can write a checkpoint (parameters, Adam moments and step count,
the batch-order generator, counters and the best parameters so far) every
few epochs and resume from it; a resumed run continues the interrupted one
bit for bit.

Usage: python -m paper_2509_01416_amd.train --out FILE [--minutes M]
           [--checkpoint FILE [--resume]]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import binding as B
from . import inputs as I

GRID = 64
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "fno2d_w32_m12_l4_g64.npy")
DEEPONET_WEIGHTS = os.path.join(WEIGHTS_DIR, "deeponet2d_h200_k100_g64.npy")


def log(msg: str):
    print(msg, flush=True)


def generate(ctx, count: int, seed0: int = 40000, chunk: int = 250):
    """Sources and solutions at p* for `count` GRF sources (device tensors)."""
    import torch
    wl = I.fno_training_set(count=count, n=GRID, seed0=seed0)
    quad = B.Quad.from_inputs(wl.quad)
    dev = "cuda"
    S = torch.empty((count, GRID, GRID), dtype=torch.float32, device=dev)
    phi = torch.zeros_like(S)
    st = torch.full((GRID, GRID), I.SIGMA_T_STAR, dtype=torch.float32, device=dev)
    ss = torch.full((GRID, GRID), I.SIGMA_S_STAR, dtype=torch.float32, device=dev)
    iters = []
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        probs = []
        for j in range(c0, c1):
            inst = wl.instances[j]
            S[j] = torch.tensor(np.asarray(inst.source, np.float32), device=dev)
            probs.append(B.Problem(sigma_t=st, sigma_s=ss, source=S[j], lx=inst.lx,
                                   ly=inst.ly, bc=inst.bc))
        rc, stats = B.tr_solve(ctx, probs, quad, None, [phi[j] for j in range(c0, c1)],
                               wl.tol, 5000)
        if rc != B.TR_OK:
            raise RuntimeError(f"training data solve returned status {rc}")
        iters += [s["iterations"] for s in stats]
        log(f"data: solved {c1}/{count} (iterations {min(iters)}..{max(iters)})")
    return S, phi


def scaled_pairs(S, phi, sa_star):
    """(S/s, sigma_a* phi / s) with s = mean |S| per instance."""
    s = S.abs().mean(dim=(1, 2), keepdim=True)
    return (S / s).contiguous(), (sa_star * phi / s).contiguous()


def rel_l2_batch(pred, target):
    d = (pred - target).double().flatten(1).norm(dim=1)
    return (d / target.double().flatten(1).norm(dim=1))


def save_checkpoint(path: str, model, rng, epoch: int, steps: int, best, hist) -> None:
    """Everything a resumed run needs to continue this one bit for bit."""
    st = model.get_state()
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=st["params"], adam_m=st["adam_m"], adam_v=st["adam_v"],
             step=np.int64(st["step"]), epoch=np.int64(epoch), steps=np.int64(steps),
             rng=np.array(json.dumps(rng.bit_generator.state)),
             best_val=np.float64(best[0]), best_epoch=np.int64(best[1]),
             best_params=(best[2] if best[2] is not None
                          else np.zeros(0, dtype=np.float32)),
             hist=np.array(json.dumps(hist)))
    os.replace(tmp, path)


def load_checkpoint(path: str, model, rng):
    """Restores the model's training state and the generator; returns
    (epoch, steps, best, hist)."""
    z = np.load(path, allow_pickle=False)
    model.set_state(dict(params=z["params"], adam_m=z["adam_m"], adam_v=z["adam_v"],
                         step=int(z["step"])))
    rng.bit_generator.state = json.loads(str(z["rng"]))
    bp = z["best_params"]
    best = (float(z["best_val"]), int(z["best_epoch"]), bp if bp.size else None)
    return int(z["epoch"]), int(z["steps"]), best, json.loads(str(z["hist"]))


def train(out_path: str, minutes: float = 3.0, count: int = 2000, n_val: int = 200,
          batch: int = 32, lr: float = 1e-3, seed: int = 1234, max_epochs: int = 100000,
          checkpoint: str = None, checkpoint_every: int = 50, resume: bool = False,
          arch: str = "fno"):
    import torch
    torch.cuda.set_device(0)
    ctx = B.Context()
    t0 = time.time()
    S, phi = generate(ctx, count)
    sa_star = I.SIGMA_T_STAR - I.SIGMA_S_STAR
    x, y = scaled_pairs(S, phi, sa_star)
    t_data = time.time() - t0
    n_tr = count - n_val
    xtr, ytr, xva, yva = x[:n_tr], y[:n_tr], x[n_tr:], y[n_tr:]
    init = _init_params(seed) if arch == "fno" else _init_deeponet(seed)
    model = B.Model(ctx, init, arch=arch)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    best = (float("inf"), 0, None)   # (validation rel L2, epoch, parameters)
    eval_every = 5
    t1 = time.time()
    epoch = 0
    steps = 0
    if resume and checkpoint and os.path.exists(checkpoint):
        epoch, steps, best, hist = load_checkpoint(checkpoint, model, rng)
        log(f"resumed from {checkpoint} at epoch {epoch} ({steps} steps)")
    while epoch < max_epochs and (time.time() - t1) < minutes * 60.0:
        perm = torch.tensor(rng.permutation(n_tr), device="cuda")
        tot = 0.0
        nb = 0
        for b0 in range(0, n_tr, batch):
            idx = perm[b0:b0 + batch]
            xb = xtr.index_select(0, idx).contiguous()
            yb = ytr.index_select(0, idx).contiguous()
            tot += model.train_step(xb, yb, lr) * idx.numel()
            nb += idx.numel()
            steps += 1
        epoch += 1
        train_mse = tot / nb
        if epoch % eval_every == 0:
            pv = model.forward(xva)
            vm = float(rel_l2_batch(pv, yva).mean())
            hist.append(dict(epoch=epoch, train_mse=train_mse, val_rel_l2_mean=vm,
                             seconds=time.time() - t1))
            if vm < best[0]:
                best = (vm, epoch, model.get_params())
            if epoch % (10 * eval_every) == 0:
                log(f"epoch {epoch}: train mse {train_mse:.3e}, validation rel L2 "
                    f"{vm:.3e}, best {best[0]:.3e} at {best[1]} ({time.time() - t1:.0f} s)")
        if checkpoint and epoch % checkpoint_every == 0:
            save_checkpoint(checkpoint, model, rng, epoch, steps, best, hist)
    if best[2] is not None:
        model.set_params(best[2])
    pv = model.forward(xva)
    val = rel_l2_batch(pv, yva)
    params = model.get_params()
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    np.save(out_path, params)
    layout = (dict(arch="fno", width=32, modes=12, layers=4, grid=GRID, params=int(params.size))
              if arch == "fno" else
              dict(arch="deeponet", sensors=GRID * GRID, hidden=200, basis=100, grid=GRID,
                   params=int(params.size)))
    meta = dict(layout=layout,
                training=dict(count=count, n_train=n_tr, n_val=n_val, batch=batch, lr=lr,
                              optimizer="Adam(0.9, 0.999, 1e-8)", epochs=epoch, steps=steps,
                              seed=seed, source_seeds=f"40000..{40000 + count - 1}",
                              sigma_t_star=I.SIGMA_T_STAR, sigma_s_star=I.SIGMA_S_STAR,
                              quadrature="level-symmetric S8", data_tol=1e-7,
                              operands="bf16 (fp32 accumulate, fp32 master weights)",
                              checkpoint=f"best validation mean rel L2, epoch {best[1]}"),
                seconds=dict(data=t_data, train=time.time() - t1),
                validation=dict(rel_l2_mean=float(val.mean()), rel_l2_max=float(val.max()),
                                rel_l2_median=float(val.median())),
                history=hist[::max(1, len(hist) // 400)])
    with open(os.path.splitext(out_path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"saved {out_path}: {epoch} epochs, {steps} steps, validation rel L2 mean "
        f"{float(val.mean()):.3e} (max {float(val.max()):.3e})")
    model.close()
    ctx.close()
    return meta


def _init_params(seed: int) -> np.ndarray:
    """Seeded initialisation (same law as the usual defaults): linear layers
    U(-1/sqrt(fan_in), +1/sqrt(fan_in)); spectral weights (1/w^2) U[0, 1)
    for the real and imaginary parts."""
    w, m, L, proj = 32, 12, 4, 128
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []

    def lin(fi, fo):
        k = 1.0 / np.sqrt(fi)
        return [rng.uniform(-k, k, size=fi * fo), rng.uniform(-k, k, size=fo)]
    parts += lin(3, w)
    for _ in range(L):
        parts.append(rng.uniform(size=2 * m * m * w * w * 2) / (w * w))
        parts += lin(w, w)
    parts += lin(w, proj)
    parts += lin(proj, 1)
    return np.concatenate(parts).astype(np.float32)


def _init_deeponet(seed: int) -> np.ndarray:
    """Seeded initialisation of the DeepONet (branch [4096, 200, 200, 100],
    trunk [2, 200, 200, 100]): every weight and bias U(-1/sqrt(fan_in),
    +1/sqrt(fan_in)), fan_in the input width of its layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fi, fo in ((GRID * GRID, 200), (200, 200), (200, 100), (2, 200), (200, 200), (200, 100)):
        k = 1.0 / np.sqrt(fi)
        parts += [rng.uniform(-k, k, size=fi * fo), rng.uniform(-k, k, size=fo)]
    return np.concatenate(parts).astype(np.float32)


def load_weights(path=None, arch: str = "fno") -> np.ndarray:
    """Trained parameters (float32 vector) written by train(); the packaged
    file of the network `arch` ("fno" or "deeponet") when path is None."""
    if path is None:
        path = DEFAULT_WEIGHTS if arch == "fno" else DEEPONET_WEIGHTS
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path}: no trained network (run "
                                "`python -m paper_2509_01416_amd.train`)")
    p = np.load(path)
    if p.dtype != np.float32 or p.ndim != 1:
        raise ValueError(f"{path}: expected a float32 vector")
    return p


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--arch", choices=("fno", "deeponet"), default="fno")
    ap.add_argument("--out", default=None)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--minutes", type=float, default=3.0)
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--max-epochs", type=int, default=100000)
    ap.add_argument("--checkpoint", default=None,
                    help="write the training state here every --checkpoint-every epochs")
    ap.add_argument("--checkpoint-every", type=int, default=50)
    ap.add_argument("--resume", action="store_true",
                    help="continue from --checkpoint if it exists")
    a = ap.parse_args(argv)
    out = a.out or (DEFAULT_WEIGHTS if a.arch == "fno" else DEEPONET_WEIGHTS)
    train(out, minutes=a.minutes, count=a.count, max_epochs=a.max_epochs, lr=a.lr, batch=a.batch,
          checkpoint=a.checkpoint, checkpoint_every=a.checkpoint_every, resume=a.resume,
          arch=a.arch)


if __name__ == "__main__":
    main()
