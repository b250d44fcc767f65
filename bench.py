#!/usr/bin/env python3
"""Benchmark of the S_N source-iteration hot path on one MI355X.

Workload (default): 16 instances of 256 x 256 cells on a 10 x 10 mfp square,
level-symmetric S16 (144 directions), two-region sigma_t in {1, 5} split by a
seeded random line, c = 0.99, Gaussian-random-field sources, vacuum faces,
tolerance 1e-6 under the error-bound stopping rule (the estimated distance
r rho / (1 - rho) to the fixed point from the change over 16 iterations; the
plain change rule, --stop change, leaves about 7e-5 at this contraction
rate).  One step = one pass of the hot
path over the batch: the equation-recast guess from the trained operator
network (Eq. 24 on the 64 x 64 network grid, block-averaged inputs, bilinear
resampling back to 256 x 256), then the source iteration to tolerance started
from that guess.  The same number of zero-start solves is timed beside it
(--zero-only times the zero-start solve alone).

Prints one JSON line: the metric (cell-angle updates/s over the whole step),
the warm/zero wall times and iteration counts, the distance of the answers
to the oracle's fixed point (stored FP64 references of three instances), the
dominant kernel's roofline from HIP events recorded live on the library
stream, the network forward's matrix-core throughput, and the FP64 oracle on
the host cores (all instances to the same tolerance on every core, one
instance for a bounded number of iterations on one core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# published FP32 vector peak (packed FP32: two operations per lane and cycle)
VALU_FP32_PEAK_TFLOPS = 157.3
# the same without packed FP32, which this library does not use: 256 CU x 4
# SIMD x 16 lanes x 2.4 GHz x 2 flop (FMA) = 78.6 TFLOP/s
VALU_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# algorithmic work of one diamond-difference cell-angle update, an FMA
# counted as two operations and the reciprocal as one: 2 FMA numerator (4),
# denominator add (1), reciprocal (1), product (1), 2 FMA outgoing faces
# (4), weighted accumulation FMA (2) = 13 flop
FLOP_PER_UPDATE = 13
# a recast tolerance near the networks' own error on the 64 x 64 families
LOOSE_RECAST_TOL = 3e-2
# algorithmic HBM bytes per cell per source iteration: read sigma_t, sigma_s,
# q, phi_old; write phi_new (FP32)
BYTES_PER_CELL_ITER = 20
# HBM bytes per sweep launch on the default workload (all 16 instances
# active) from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by what the counters
# read for a 256 MiB elementwise copy (profiles/sweep2d_fast_two_region_16x256_S16.md);
# valid only for the kernel source with this hash prefix (sweep_source_hash),
# otherwise null
SWEEP_TRAFFIC_BYTES = 79.82e6
SWEEP_TRAFFIC_SRC = "ba5aeb282ea67ddd"


def sweep_source_hash() -> str:
    """Hash prefix of the sweep kernel's source (the kernel file and the
    device header it includes)."""
    h = hashlib.sha256()
    for f in ("sweep2d.hip", "common.h"):
        h.update(open(os.path.join(ROOT, "paper_2509_01416_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=16)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--stop", choices=("bound", "change"), default="bound",
                    help="stopping rule of the source iteration")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the one-core oracle sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB fill and copy (counter calibration)")
    ap.add_argument("--zero-only", action="store_true",
                    help="time the zero-start source iteration alone")
    ap.add_argument("--max-iter", type=int, default=20000,
                    help="cap on source iterations per solve (profiling runs)")
    ap.add_argument("--recast-tol", type=float, default=1e-3,
                    help="recast-loop tolerance (above the BF16 network's change floor)")
    ap.add_argument("--recast-max", type=int, default=30)
    ap.add_argument("--no-eigen", action="store_true",
                    help="skip the k-eigenvalue measurements")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the uneven-batch and network-grid legs")
    ap.add_argument("--network-only", action="store_true",
                    help="time the networks alone and print their figures (counter runs)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="run the uneven-batch leg alone and print its figures (counter runs)")
    ap.add_argument("--weights", default=None,
                    help="trained network parameters (default: the packaged file)")
    return ap.parse_args()


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, tol: float, stop: str, target_1core_s: float):
    """The FP64 C oracle on the host cores, on the same instances:
    all cores: every instance solved from zero to the same tolerance and
      stopping rule, one thread per instance (measured time to tolerance);
    one core: instance 0 for a bounded number of iterations (about
      target_1core_s), and the batch's time to tolerance on one core
      estimated from that rate and the all-core run's iteration counts."""
    import oracle
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu, len(wl.instances)))
    M = wl.quad.n_dir
    kw = dict(norm="bound", stride=16) if stop == "bound" else dict(norm="l2")
    t0 = time.perf_counter()
    res = oracle.solve_many(wl.instances, wl.quad, tol=tol, threads=threads, f32_inputs=True,
                            **kw)
    dt_all = time.perf_counter() - t0
    its = [int(r.iterations) for r in res]
    ups_all = sum(n * i.cells for n, i in zip(its, wl.instances)) * M
    inst = wl.instances[0]
    t0 = time.perf_counter()
    oracle.solve_instance(inst, wl.quad, tol=1e-300, max_iter=2)
    per_it = (time.perf_counter() - t0) / 2
    n1 = int(max(2, min(5000, target_1core_s / max(per_it, 1e-6))))
    t0 = time.perf_counter()
    r1 = oracle.solve_instance(inst, wl.quad, tol=1e-300, max_iter=n1)
    dt1 = time.perf_counter() - t0
    rate1 = r1.iterations * inst.cells * M / dt1
    return {"value": ups_all / dt_all, "unit": "cell-angle updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"all {len(wl.instances)} instances from zero to {tol:g} ({stop} rule), "
                      f"one thread per instance, {dt_all:.1f} s wall; one core: instance 0 "
                      f"for {n1} iterations, {dt1:.1f} s",
            "cpu_model": _cpu_model(), "host_cpus": ncpu,
            "cores_all": {"threads": threads, "seconds_to_tolerance": dt_all,
                          "updates_per_s": ups_all / dt_all},
            "cores_1": {"updates_per_s": rate1,
                        "seconds_to_tolerance_estimated": ups_all / rate1},
            "oracle_iterations_zero_start": its,
            "sinusoid_128": cpu_sinusoid(tol, stop)}


def cpu_sinusoid(tol: float, stop: str):
    """The FP64 C oracle on one core for the 128 x 128 sinusoidal problem,
    from zero to the same tolerance and stopping rule (a fraction of a
    second of host work)."""
    import oracle
    from paper_2509_01416_amd import inputs as I
    wl = I.sinusoid_128()
    kw = dict(norm="bound", stride=16) if stop == "bound" else dict(norm="l2")
    t0 = time.perf_counter()
    r = oracle.solve_instance(wl.instances[0], wl.quad, tol=tol, f32_inputs=True, **kw)
    dt = time.perf_counter() - t0
    ups = r.iterations * wl.instances[0].cells * wl.quad.n_dir
    return {"threads": 1, "seconds_to_tolerance": dt, "iterations": int(r.iterations),
            "updates_per_s": ups / dt}


# algorithmic FLOP of one network forward per 64 x 64 sample (dense products
# as performed: DFT products, per-mode complex mixing, pointwise layers, lift
# and projection)
def fno_flop_per_sample(n=64, w=32, m=12, layers=4, proj=128):
    P = n * n
    dft = 2 * (n * 2 * m * n + 4 * m * m * 2 * n + 2 * n * m * 4 * m + n * n * 2 * m) * w
    mix = 2 * m * m * w * w * 8
    point = 2 * w * P * w
    return 2 * 3 * w * P + layers * (dft + mix + point) + 2 * proj * P * w + 2 * proj * P


BF16_MFMA_PEAK_TFLOPS = 2500.0


def rel_l2_vs_refs(args, warm, zero, torch):
    """Relative L2 distance of the warm- and zero-start answers to the stored
    FP64 oracle references (instances 0, 7, 15 of the default workload;
    None for other workloads)."""
    if args.instances != 16 or args.n != 256:
        return None
    z = np.load(os.path.join(ROOT, "tests", "golden", "two_region_16x256_S16_refs.npz"))
    out = {"instances": [int(k) for k in z["index"]], "reference": "FP64 oracle to a "
           "relative change of 1e-11 on the FP32-rounded fields"}
    for name, phis in (("warm", warm), ("zero", zero)):
        if name == "warm" and args.zero_only:
            continue
        e = []
        for k, ref in zip(z["index"], z["phi"]):
            ref = ref.astype(np.float64)
            got = phis[int(k)].cpu().numpy().astype(np.float64)
            e.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        out[name] = e
        out[name + "_max"] = max(e)
    return out


def uneven_leg(B, I, torch, args):
    """The 256-instance uneven batch (sides 32..128, 4 x 4-block sigma_t,
    c in [0.5, 0.95], S8) solved from zero in one batched call, on its own
    context (the planner's launch shape): median wall time of three solves,
    cell-angle updates/s, and the sweep kernel's time per launch."""
    wl = I.batched_uneven(256)
    f = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    probs = [B.Problem(sigma_t=f(i.sigma_t), sigma_s=f(i.sigma_s), source=f(i.source),
                       lx=i.lx, ly=i.ly) for i in wl.instances]
    quad = B.Quad.from_inputs(wl.quad)
    phis = [torch.zeros_like(p.sigma_t) for p in probs]
    ctx = B.Context()
    ctx.set_stop_rule(args.stop)
    plan = ctx.sweep_plan(probs, quad)
    B.tr_solve(ctx, probs, quad, None, phis, args.tol, args.max_iter)   # warm-up
    times, ups = [], 0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = B.tr_solve(ctx, probs, quad, None, phis, args.tol, args.max_iter)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ups = sum(s["iterations"] * i.cells for s, i in zip(st, wl.instances)) * wl.quad.n_dir
    ctx.profile(True)
    B.tr_solve(ctx, probs, quad, None, phis, args.tol, args.max_iter)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    med = float(np.median(times))
    its = [s["iterations"] for s in st]
    log(f"[bench] uneven batch: {med * 1e3:.1f} ms, {ups / med:.3e} updates/s")
    # sweep roofline of the profiled solve: its updates (the same iteration
    # counts) at FLOP_PER_UPDATE each over the summed sweep kernel time
    sweep_s = prof["sweep_ms"] * 1e-3
    achieved = ups * FLOP_PER_UPDATE / sweep_s / 1e12 if sweep_s > 0 else None
    return {"workload": wl.name, "ms": med * 1e3, "status": rc,
            "cell_angle_updates_per_s": ups / med, "iterations_min_max": [min(its), max(its)],
            "iterations_mean": float(np.mean(its)),
            "sweep_plan": plan,
            "sweep_ms_per_launch": prof["sweep_ms"] / max(1, prof["sweep_launches"]),
            "sweep_launches": prof["sweep_launches"],
            "sweep_roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_FP32_PEAK_TFLOPS,
                               "unit": "TFLOP/s",
                               "frac": achieved / VALU_FP32_PEAK_TFLOPS if achieved else None}}


def sinusoid_leg(B, I, torch, args):
    """The 128 x 128 sinusoidal problem (S8, sigma_t = 1 + 0.5 sin sin,
    c = 0.9, GRF source, vacuum) solved from zero on its own context, launch
    shape by the autotuner (outside the timing): median wall time of five
    solves, cell-angle updates/s, iteration count, the sweep's time per
    launch, and the distance to the stored FP64 oracle reference."""
    wl = I.sinusoid_128()
    inst = wl.instances[0]
    f = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    probs = [B.Problem(sigma_t=f(inst.sigma_t), sigma_s=f(inst.sigma_s), source=f(inst.source),
                       lx=inst.lx, ly=inst.ly)]
    quad = B.Quad.from_inputs(wl.quad)
    phis = [torch.zeros_like(probs[0].sigma_t)]
    ctx = B.Context()
    ctx.set_stop_rule(args.stop)
    tuned = ctx.autotune(probs, quad)
    B.tr_solve(ctx, probs, quad, None, phis, wl.tol, args.max_iter)   # warm-up
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = B.tr_solve(ctx, probs, quad, None, phis, wl.tol, args.max_iter)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ctx.profile(True)
    B.tr_solve(ctx, probs, quad, None, phis, wl.tol, args.max_iter)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    med = float(np.median(times))
    its = int(st[0]["iterations"])
    ups = its * inst.cells * wl.quad.n_dir
    z = np.load(os.path.join(ROOT, "tests", "golden", "sinusoid_128_S8_ref.npz"))
    ref = z["phi"].astype(np.float64)
    got = phis[0].cpu().numpy().astype(np.float64)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    log(f"[bench] sinusoid 128^2: {med * 1e3:.2f} ms, {its} iterations, "
        f"{ups / med:.3e} updates/s, rel L2 vs oracle {e:.2e}")
    return {"workload": wl.name, "ms": med * 1e3, "status": rc,
            "cell_angle_updates_per_s": ups / med, "iterations": its,
            "oracle_iterations_same_rule": int(z["iters_bound"] if args.stop == "bound"
                                               else z["iters_change"]),
            "sweep_plan": {k: v for k, v in tuned.items() if k != "ms"},
            "sweep_ms_per_launch": prof["sweep_ms"] / max(1, prof["sweep_launches"]),
            "rel_l2_vs_oracle": e}


def network_grid_leg(models, B, I, torch, args):
    """Warm start against zero start on the network's own 64 x 64 grid (the
    sinusoidal and random-line families, 64 instances each, S8), for each
    trained network: wall time of the whole step (recast guess + source
    iteration) against the zero-start solve, medians of five, with
    iteration counts (own context: the planner's launch shape), at the
    benchmark's recast tolerance and at a looser one.  These
    families contract at rates up to about 0.9, where the plain change rule
    at 1e-6 stays within about 1e-5 of the fixed point; the error-bound
    rule's 16-iteration test stride would round their 25-65 iterations up
    to multiples of 16, so the plain rule is used here."""
    out = {}
    ctx = B.Context()
    ctx.set_stop_rule("change")
    for arch, model in models.items():
        out[arch] = _network_grid_arch(ctx, model, B, I, torch, args)
    out["workload"] = "fno_eval families, 64 x 64 instances, S8"
    ctx.close()
    return out


def _network_grid_arch(ctx, model, B, I, torch, args):
    out = {}
    f = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    for family in ("sinusoid", "line"):
        wl = I.fno_eval_set(family, count=64)
        probs = [B.Problem(sigma_t=f(i.sigma_t), sigma_s=f(i.sigma_s), source=f(i.source),
                           lx=i.lx, ly=i.ly) for i in wl.instances]
        quad = B.Quad.from_inputs(wl.quad)
        phis = [torch.zeros_like(p.sigma_t) for p in probs]

        def zero():
            return B.tr_solve(ctx, probs, quad, None, phis, args.tol, args.max_iter)[1], None

        def warm_at(rtol):
            def warm():
                _, sg = B.no_recast_guess(ctx, model, probs, I.SIGMA_T_STAR, I.SIGMA_S_STAR,
                                          rtol, args.recast_max, phis)
                return B.tr_solve(ctx, probs, quad, phis, phis, args.tol, args.max_iter)[1], sg
            return warm

        def run(fn, reps=5):
            fn()
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, sg = fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            r = {"ms": float(np.median(ts)) * 1e3,
                 "si_iterations_mean": float(np.mean([s["iterations"] for s in st])),
                 "si_iterations_max": int(max(s["iterations"] for s in st))}
            if sg is not None:
                r["recast_iterations_mean"] = float(np.mean([s["iterations"] for s in sg]))
                r["recast_iterations_max"] = int(max(s["iterations"] for s in sg))
            return r
        res = {}
        z = run(zero)
        w = run(warm_at(args.recast_tol))
        res["zero_ms"] = z["ms"]
        res["zero_si_iterations_mean"] = z["si_iterations_mean"]
        res["zero_si_iterations_max"] = z["si_iterations_max"]
        res["warm_ms"] = w["ms"]
        res["warm_si_iterations_mean"] = w["si_iterations_mean"]
        res["warm_si_iterations_max"] = w["si_iterations_max"]
        res["recast_iterations_mean"] = w["recast_iterations_mean"]
        res["recast_iterations_max"] = w["recast_iterations_max"]
        res["time_reduction"] = 1.0 - w["ms"] / z["ms"]
        # the guess barely improves below the network's own error on these
        # families: the same step with a looser recast tolerance
        loose = run(warm_at(LOOSE_RECAST_TOL))
        loose["recast_tol"] = LOOSE_RECAST_TOL
        loose["time_reduction"] = 1.0 - loose["ms"] / z["ms"]
        res["loose_recast"] = loose
        out[family] = res
        log(f"[bench] 64^2 {family}: warm {res['warm_ms']:.2f} ms (tol {LOOSE_RECAST_TOL:g}: "
            f"{loose['ms']:.2f} ms), zero {res['zero_ms']:.2f} ms")
    return out


def eigen_leg(ctx, model, B, I, torch, args, don=None):
    """k-eigenvalue measurements (section 5.2-5.3, Appendix A2), tolerance
    1e-4 on k, the flux and the inner solves (the paper's uniform
    criterion): the model-based power iteration on 16 x 256^2 S16 (the x-y
    eigen Case 1 analogue), the three-group problem of Tables 8-9 on
    16 x 256^2 S16, and on the network's 64 x 64 grid the model-based solve
    beside SP and CP (network loop, then model-based refinement) with the
    FNO and with the DeepONet, as wall times normalised to the model-based
    one."""
    dev = "cuda"
    f = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)

    def batch(wl):
        probs = [B.Problem(sigma_t=f(i.sigma_t), sigma_s=f(i.sigma_s), source=None,
                           lx=i.lx, ly=i.ly) for i in wl.instances]
        return probs, [f(a) for a in wl.extra["nu_sigma_f"]], B.Quad.from_inputs(wl.quad)

    spread = {}

    def wall(fn, reps, name):
        # median of reps solves: an isolated call in a process can take
        # two to three times the steady time (host-side stalls between the
        # read-backs), and a mean of few calls would report that instead
        times, r = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        spread[name] = [round(min(times), 2), round(max(times), 2)]
        return float(np.median(times)), r

    tol = 1e-4
    wl = I.eigen_case1_2d(16, 256)
    probs, nsf, quad = batch(wl)
    phis = [torch.zeros_like(p.sigma_t) for p in probs]
    run = lambda: B.tr_eigen(ctx, probs, nsf, quad, None, phis, None, tol, tol, tol, 500, 20000)
    run()
    ms, (rc, st) = wall(run, 5, "model_based_256")
    M = wl.quad.n_dir
    sweeps = sum(s["inner"] * i.cells for s, i in zip(st, wl.instances)) * M
    big = {"workload": wl.name, "ms": ms, "status": rc,
           "k_mean": float(np.mean([s["k"] for s in st])),
           "outer_mean": float(np.mean([s["outer"] for s in st])),
           "inner_sweeps_mean": float(np.mean([s["inner"] for s in st])),
           "cell_angle_updates_per_s": sweeps / (ms * 1e-3),
           "balance_rel_max": float(max(s["balance_rel"] for s in st))}
    log(f"[bench] eigen {wl.name}: {ms:.1f} ms k={big['k_mean']:.5f} "
        f"outer={big['outer_mean']:.1f} inner={big['inner_sweeps_mean']:.0f}")

    wl = I.three_group_2d(16, 256)
    mgp = [B.Problem(sigma_t=f(i.sigma_t), sigma_s=None, source=None, lx=i.lx, ly=i.ly)
           for i in wl.instances]
    mgd = [dict(sigma_t=[f(a) for a in gd["sigma_t"]],
                sigma_s=[[None if a is None else f(a) for a in row] for row in gd["sigma_s"]],
                nu_sigma_f=[f(a) for a in gd["nu_sigma_f"]], chi=gd["chi"])
           for gd in wl.extra["groups"]]
    mgo = [[torch.zeros_like(p.sigma_t) for _ in range(3)] for p in mgp]
    qmg = B.Quad.from_inputs(wl.quad)
    run = lambda: B.tr_eigen_mg(ctx, mgp, mgd, qmg, None, mgo, None, tol, tol, tol, 500, 20000)
    run()
    ms, (rc, st) = wall(run, 5, "three_group_256")
    sweeps = sum(s["inner"] * i.cells for s, i in zip(st, wl.instances)) * wl.quad.n_dir
    three = {"workload": wl.name, "ms": ms, "status": rc,
             "k_mean": float(np.mean([s["k"] for s in st])),
             "outer_mean": float(np.mean([s["outer"] for s in st])),
             "inner_sweeps_mean": float(np.mean([s["inner"] for s in st])),
             "cell_angle_updates_per_s": sweeps / (ms * 1e-3),
             "balance_rel_max": float(max(s["balance_rel"] for s in st))}
    log(f"[bench] eigen {wl.name}: {ms:.1f} ms k={three['k_mean']:.5f} "
        f"outer={three['outer_mean']:.1f} inner={three['inner_sweeps_mean']:.0f}")
    del mgp, mgd, mgo

    wl = I.eigen_sine_64(16)
    probs, nsf, quad = batch(wl)
    phis = [torch.zeros_like(p.sigma_t) for p in probs]
    mb = lambda: B.tr_eigen(ctx, probs, nsf, quad, None, phis, None, tol, tol, tol, 500, 20000)
    sp = lambda: B.eigen_preconditioned(ctx, model, probs, nsf, quad, I.SIGMA_T_STAR,
                                        I.SIGMA_S_STAR, B.NO_EIGEN_SP, phis, tol, tol, tol)
    cp = lambda: B.eigen_preconditioned(ctx, model, probs, nsf, quad, I.SIGMA_T_STAR,
                                        I.SIGMA_S_STAR, B.NO_EIGEN_CP, phis, tol, tol, tol)
    small = {"workload": wl.name}
    legs = [("model_based", mb), ("sp", sp), ("cp", cp)]
    if don is not None:
        legs += [(name, (lambda v: lambda: B.eigen_preconditioned(
                    ctx, don, probs, nsf, quad, I.SIGMA_T_STAR, I.SIGMA_S_STAR, v, phis,
                    tol, tol, tol))(v))
                 for name, v in (("deeponet_sp", B.NO_EIGEN_SP), ("deeponet_cp", B.NO_EIGEN_CP))]
    for name, fn in legs:
        fn()
        ms, r = wall(fn, 5, name)
        if name == "model_based":
            rc, st = r
            small[name] = {"ms": ms, "status": rc, "k_mean": float(np.mean([s["k"] for s in st])),
                           "inner_sweeps_mean": float(np.mean([s["inner"] for s in st]))}
        else:
            rc, st_no, st = r
            small[name] = {"ms": ms, "status": rc,
                           "k_mean": float(np.mean([s["k"] for s in st])),
                           "network_k_mean": float(np.mean([s["k"] for s in st_no])),
                           "network_outer_mean": float(np.mean([s["outer"] for s in st_no])),
                           "refine_inner_sweeps_mean": float(np.mean([s["inner"] for s in st]))}
        log(f"[bench] eigen {wl.name} {name}: {ms:.1f} ms")
    base = small["model_based"]["ms"]
    for name in small:
        if name not in ("workload", "model_based"):
            small[name]["normalised_time_pct"] = 100.0 * small[name]["ms"] / base
    return {"tol": tol, "timing": "median of 5 solves after one warm-up",
            "min_max_ms": spread, "model_based_256": big, "three_group_256": three,
            "preconditioned_64": small}


def _forward_ms(ctx, model, nb, torch, reps=20):
    """Mean forward time of a batch of nb 64 x 64 fields, HIP events on the
    library stream."""
    xin = torch.randn(nb, 64, 64, device="cuda")
    xout = torch.empty_like(xin)
    for _ in range(3):
        model.forward(xin, xout)
    s = ctx.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        model.forward(xin, xout)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def network_leg(ctx, model, don, nb, torch):
    """Network forwards on the recast batch (nb fields of 64 x 64) and on 64
    fields (the 64 x 64 families), for the FNO and the DeepONet, and one FNO
    training step at batch 32 (forward, MSE, backward, Adam, loss
    read-back; lr = 0 leaves the parameters as they are)."""
    fwd_ms = _forward_ms(ctx, model, nb, torch)
    fl = fno_flop_per_sample() * nb
    out = {"forward_ms": fwd_ms, "batch": nb, "flop_per_sample": fno_flop_per_sample(),
           "achieved_TFLOPs": fl / (fwd_ms * 1e-3) / 1e12,
           "peak_TFLOPs": BF16_MFMA_PEAK_TFLOPS,
           "frac": fl / (fwd_ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS,
           "dtype": "bf16 operands, fp32 accumulate",
           "forward_ms_batch64": _forward_ms(ctx, model, 64, torch)}
    if don is not None:
        out["deeponet_forward_ms"] = _forward_ms(ctx, don, nb, torch)
        out["deeponet_forward_ms_batch64"] = _forward_ms(ctx, don, 64, torch)
    tb = 32
    tin = torch.randn(tb, 64, 64, device="cuda")
    tgt = torch.randn(tb, 64, 64, device="cuda")
    for _ in range(2):
        model.train_step(tin, tgt, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    treps = 10
    for _ in range(treps):
        model.train_step(tin, tgt, 0.0)
    torch.cuda.synchronize()
    out["train_step_ms"] = (time.perf_counter() - t0) * 1e3 / treps
    out["train_batch"] = tb
    return out


def network_only(args):
    """--network-only: the network leg alone (for counter runs)."""
    import torch
    from paper_2509_01416_amd import binding as B
    from paper_2509_01416_amd import train as T
    ctx = B.Context()
    model = B.Model(ctx, T.load_weights(args.weights))
    don = B.Model(ctx, T.load_weights(arch="deeponet"), arch="deeponet")
    net = network_leg(ctx, model, don, args.instances, torch)
    print(json.dumps({"network": net}), flush=True)
    ctx.close()


def uneven_only(args):
    """--uneven-only: the uneven-batch leg alone (for counter runs)."""
    import torch
    from paper_2509_01416_amd import binding as B
    from paper_2509_01416_amd import inputs as I
    print(json.dumps({"uneven_batch_256": uneven_leg(B, I, torch, args)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this "
              "build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.uneven_only:
        uneven_only(args)
        return
    if args.network_only:
        network_only(args)
        return
    import torch
    from paper_2509_01416_amd import binding as B
    from paper_2509_01416_amd import inputs as I
    from paper_2509_01416_amd import train as T
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    wl = I.hard_two_region(args.instances, args.n)
    quad = B.Quad.from_inputs(wl.quad)
    M = wl.quad.n_dir
    log(f"[bench] workload {wl.name}: {len(wl.instances)} x {args.n}^2, M={M}")
    dev = "cuda"
    probs = [B.Problem(sigma_t=torch.tensor(i.sigma_t, dtype=torch.float32, device=dev),
                       sigma_s=torch.tensor(i.sigma_s, dtype=torch.float32, device=dev),
                       source=torch.tensor(i.source, dtype=torch.float32, device=dev),
                       lx=i.lx, ly=i.ly) for i in wl.instances]
    phis = [torch.zeros_like(p.sigma_t) for p in probs]
    phis0 = [torch.zeros_like(p.sigma_t) for p in probs]
    ctx = B.Context()
    ctx.set_stop_rule(args.stop)
    planned = ctx.sweep_plan(probs, quad)
    t_tune = time.perf_counter()
    tuned = ctx.autotune(probs, quad, reps=3)
    t_tune = time.perf_counter() - t_tune
    plan = ctx.sweep_plan(probs, quad)
    log(f"[bench] planner {planned}; autotuned {tuned} in {t_tune:.2f} s")
    model = None if args.zero_only else B.Model(ctx, T.load_weights(args.weights))

    def zero_step():
        rc, st = B.tr_solve(ctx, probs, quad, None, phis0, args.tol, args.max_iter)
        return st, None, 0.0

    def warm_step():
        t0 = time.perf_counter()
        rcg, sg = B.no_recast_guess(ctx, model, probs, I.SIGMA_T_STAR, I.SIGMA_S_STAR,
                                    args.recast_tol, args.recast_max, phis)
        tg = time.perf_counter() - t0
        rc, st = B.tr_solve(ctx, probs, quad, phis, phis, args.tol, args.max_iter)
        return st, sg, tg

    def timed(step, k, profile):
        if profile:
            ctx.profile(True)
        updates, its, rits, tg = 0, [], [], 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            st, sg, g = step()
            its.append([s["iterations"] for s in st])
            if sg is not None:
                rits.append([s["iterations"] for s in sg])
            tg += g
            updates += sum(s["iterations"] * i.cells for s, i in zip(st, wl.instances)) * M
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read() if profile else None
        if profile:
            ctx.profile(False)
        return dict(updates=updates, dt=dt, its=its, rits=rits, guess_s=tg, prof=prof)

    step = zero_step if args.zero_only else warm_step
    result = phis0 if args.zero_only else phis
    for w in range(args.warmup):
        st, sg, _ = step()
        log(f"[bench] warmup {w}: iterations {[s['iterations'] for s in st][:4]}...")
        if not args.zero_only:
            zero_step()
    # the timed runs record no events; kernel durations come from a
    # separate profiled step
    main_run = timed(step, args.steps, False)
    log(f"[bench] {args.steps} steps in {main_run['dt']:.3f} s")
    zero_run = main_run if args.zero_only else timed(zero_step, args.steps, False)
    log(f"[bench] zero start: {args.steps} steps in {zero_run['dt']:.3f} s")
    prof_run = timed(step, 1, True)
    prof = prof_run["prof"]
    log(f"[bench] profiled step: {prof}")

    accuracy = rel_l2_vs_refs(args, result, phis0, torch)
    log(f"[bench] distance to the oracle's fixed point: {accuracy}")

    updates, dt = main_run["updates"], main_run["dt"]
    ms_step = dt * 1e3 / args.steps
    sweep_ms = prof["sweep_ms"]
    flops = prof_run["updates"] * FLOP_PER_UPDATE
    achieved = flops / (sweep_ms * 1e-3) / 1e12 if sweep_ms > 0 else None
    cell_iters = prof_run["updates"] / M
    hbm = cell_iters * BYTES_PER_CELL_ITER / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    traffic = None
    default_wl = args.instances == 16 and args.n == 256
    if default_wl and sweep_source_hash() == SWEEP_TRAFFIC_SRC:
        traffic = SWEEP_TRAFFIC_BYTES
    roof = {"bound": "alu", "achieved": achieved, "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / VALU_FP32_PEAK_TFLOPS if achieved else None,
            "flop_per_update": FLOP_PER_UPDATE,
            "frac_vs_nonpacked_peak": (achieved / VALU_FP32_NONPACKED_TFLOPS
                                       if achieved else None),
            "nonpacked_peak": VALU_FP32_NONPACKED_TFLOPS,
            "traffic": traffic, "traffic_unit": "bytes per launch",
            "kernel": "sweep2d_fast_kernel" if plan.get("specialised") else "sweep2d_kernel",
            "avg_launch_ms": sweep_ms / max(1, prof["sweep_launches"]),
            "launches": prof["sweep_launches"],
            "hbm_algorithmic_GBs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS if hbm else None}

    network = None
    don = None if model is None else B.Model(ctx, T.load_weights(arch="deeponet"),
                                             arch="deeponet")
    if model is not None:
        network = network_leg(ctx, model, don, len(probs), torch)
    eigen = None
    if model is not None and not args.no_eigen:
        eigen = eigen_leg(ctx, model, B, I, torch, args, don)
    uneven = None if args.no_extra else uneven_leg(B, I, torch, args)
    sinus = None if args.no_extra else sinusoid_leg(B, I, torch, args)
    netgrid = (None if args.no_extra or model is None
               else network_grid_leg({"fno": model, "deeponet": don}, B, I, torch, args))
    don_step = None
    if don is not None and not args.no_extra:
        # the headline batch with the DeepONet's recast guess (same rule)
        def don_warm():
            t0 = time.perf_counter()
            _, sg = B.no_recast_guess(ctx, don, probs, I.SIGMA_T_STAR, I.SIGMA_S_STAR,
                                      args.recast_tol, args.recast_max, phis)
            tg = time.perf_counter() - t0
            _, st = B.tr_solve(ctx, probs, quad, phis, phis, args.tol, args.max_iter)
            return st, sg, tg
        don_warm()
        r = timed(don_warm, args.steps, False)
        don_step = {"warm_ms": r["dt"] * 1e3 / args.steps,
                    "recast_ms": r["guess_s"] * 1e3 / args.steps,
                    "recast_iterations_mean": float(np.mean(r["rits"][-1])),
                    "recast_ms_per_update": r["guess_s"] * 1e3 / args.steps /
                                            max(1, max(r["rits"][-1])),
                    "si_iterations_mean": float(np.mean(r["its"][-1])),
                    "si_iterations_max": int(max(r["its"][-1])),
                    "updates_per_s": r["updates"] / r["dt"],
                    "rel_l2_vs_oracle": rel_l2_vs_refs(args, phis, phis0, torch)}
        log(f"[bench] DeepONet warm step {don_step['warm_ms']:.1f} ms")

    if args.calib_copy:
        # counter calibration: a fill writing 256 MiB, then an elementwise
        # kernel reading and writing 256 MiB each
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        a.fill_(1.0)
        b = a * 1.0
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu:
        log("[bench] oracle CPU baseline ...")
        cpu = cpu_baseline(wl, args.tol, args.stop, args.cpu_seconds)
        log(f"[bench] cpu {cpu}")

    zero_ms = zero_run["dt"] * 1e3 / args.steps
    mean = lambda rows: float(np.mean(rows[-1])) if rows else None
    out = {
        "metric": "cell-angle updates/s; wall time to 1e-6 residual, NO warm start vs zero start",
        "value": updates / dt,
        "unit": "cell-angle updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "instances": len(wl.instances),
                   "grid": f"{args.n}x{args.n}", "directions": M,
                   "tol": args.tol,
                   "stop_rule": ("error bound r rho/(1-rho) over 16-iteration changes"
                                 if args.stop == "bound" else "relative L2 change"),
                   "start": "zero" if args.zero_only else "operator-network recast warm start",
                   "recast_tol": None if args.zero_only else args.recast_tol,
                   "recast_max_iter": None if args.zero_only else args.recast_max,
                   "sweep_plan": plan, "planner_choice": planned,
                   "autotune_s": t_tune},
        "warm_vs_zero": {
            "warm_ms": None if args.zero_only else ms_step,
            "zero_ms": zero_ms,
            "time_reduction": None if args.zero_only else 1.0 - ms_step / zero_ms,
            "recast_ms": None if args.zero_only else main_run["guess_s"] * 1e3 / args.steps,
            "recast_iterations_mean": mean(main_run["rits"]),
            # the batch's updates run until its slowest instance stops
            "recast_ms_per_update": (None if args.zero_only else
                                     main_run["guess_s"] * 1e3 / args.steps /
                                     max(1, max(main_run["rits"][-1]))),
            "si_iterations_mean_warm": None if args.zero_only else mean(main_run["its"]),
            "si_iterations_mean_zero": mean(zero_run["its"]),
            "si_iterations_max_warm": None if args.zero_only else int(max(main_run["its"][-1])),
            "si_iterations_max_zero": int(max(zero_run["its"][-1])),
            "zero_start_updates_per_s": zero_run["updates"] / zero_run["dt"]},
        "iterations": main_run["its"][-1],
        "rel_l2_vs_oracle": accuracy,
        "roofline": roof,
        "network": network,
        "eigen": eigen,
        "uneven_batch_256": uneven,
        "sinusoid_128": sinus,
        "warm_vs_zero_64": netgrid,
        "deeponet_warm_step": don_step,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if model is not None:
        model.close()
    if don is not None:
        don.close()
    ctx.close()


if __name__ == "__main__":
    main()
