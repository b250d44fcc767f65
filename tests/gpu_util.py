"""Helpers for the GPU tests: move seeded instances onto the device."""
import os
import sys

import numpy as np

from paper_2509_01416_amd import binding as B


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_problem(inst, torch):
    dev = "cuda"
    f = lambda a: torch.tensor(np.asarray(a, dtype=np.float32).reshape(
        (inst.nx,) if inst.dim == 1 else (inst.ny, inst.nx)), device=dev)
    s1 = getattr(inst, "sigma_s1", None)
    return B.Problem(sigma_t=f(inst.sigma_t), sigma_s=f(inst.sigma_s),
                     source=f(inst.source), lx=inst.lx, ly=inst.ly,
                     bc=tuple(inst.bc), sigma_s1=None if s1 is None else f(s1))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_inf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())
