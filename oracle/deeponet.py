"""FP64 deep operator network (DeepONet): forward, hand-derived backward.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Architecture (arXiv 2509.01416 section 4.1, Eq. 11; Appendix A1): a branch
network maps the source sampled at the sensor points to coefficients, a
trunk network maps a position to basis values, and the output at that
position is their inner product.  Both are fully connected with ReLU
between layers; the last layer of each is linear (no activation), and the
inner product carries no bias.  The paper's 1-D network has branch
[100, 200, 200, 100] and trunk [1, 200, 200, 100], 141,200 parameters.  The
x-y network keeps the hidden sizes with the 64 x 64 grid as sensors and the
cell centre (x/lx, y/ly) as trunk input: branch [4096, 200, 200, 100], trunk
[2, 200, 200, 100].

Flat parameter vector, in this order (row-major, input index first):
  W1[s][h], b1[h], W2[h][h], b2[h], W3[h][k], b3[k]        (branch)
  V1[d][h], c1[h], V2[h][h], c2[h], V3[h][k], c3[k]        (trunk)
with s sensors, d trunk inputs, h hidden units and k basis functions.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Layout:
    sensors: int = 4096
    coords: int = 2
    hidden: int = 200
    basis: int = 100

    def shapes(self):
        s, d, h, k = self.sensors, self.coords, self.hidden, self.basis
        return [("W1", (s, h)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)),
                ("W3", (h, k)), ("b3", (k,)),
                ("V1", (d, h)), ("c1", (h,)), ("V2", (h, h)), ("c2", (h,)),
                ("V3", (h, k)), ("c3", (k,))]

    def count(self) -> int:
        return int(sum(np.prod(sh) for _, sh in self.shapes()))


PAPER_1D = Layout(sensors=100, coords=1, hidden=200, basis=100)


def unpack(p: np.ndarray, L: Layout) -> dict:
    out, o = {}, 0
    for name, sh in L.shapes():
        n = int(np.prod(sh))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    assert o == p.size
    return out


def pack(d: dict, L: Layout) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1)
                           for name, _ in L.shapes()])


def init_params(L: Layout, seed: int) -> np.ndarray:
    """Linear layers U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, sh in L.shapes():
        fan_in = sh[0] if len(sh) == 2 else None
        if fan_in is None:   # bias: fan-in of the weight before it
            fan_in = prev
        k = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-k, k, size=int(np.prod(sh))))
        prev = sh[0] if len(sh) == 2 else prev
    return np.concatenate(parts)


def grid_coords(n: int) -> np.ndarray:
    """(n*n, 2) cell centres (x/lx, y/ly), cell-major with x fastest."""
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c)
    return np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)


def relu(z):
    return np.maximum(z, 0.0)


def forward(p: np.ndarray, u: np.ndarray, y: np.ndarray, L: Layout):
    """u: (B, sensors) sampled inputs, y: (P, coords) positions ->
    (out (B, P), cache)."""
    q = unpack(p, L)
    z1 = u @ q["W1"] + q["b1"]
    a1 = relu(z1)
    z2 = a1 @ q["W2"] + q["b2"]
    a2 = relu(z2)
    coef = a2 @ q["W3"] + q["b3"]                  # (B, k)
    t1 = y @ q["V1"] + q["c1"]
    g1 = relu(t1)
    t2 = g1 @ q["V2"] + q["c2"]
    g2 = relu(t2)
    basis = g2 @ q["V3"] + q["c3"]                 # (P, k)
    out = coef @ basis.T                           # Eq. 11: sum_k b_k t_k(y)
    cache = dict(u=u, y=y, z1=z1, a1=a1, z2=z2, a2=a2, coef=coef,
                 t1=t1, g1=g1, t2=t2, g2=g2, basis=basis)
    return out, cache


def backward(p: np.ndarray, cache: dict, gout: np.ndarray, L: Layout,
             parts: dict = None) -> np.ndarray:
    """Gradient of sum(gout * out) with respect to the flat parameters;
    `parts` (optional dict) also receives the gradients of the
    pre-activations (gz1, gz2, gt1, gt2) and of coef and basis."""
    q = unpack(p, L)
    g = {}
    gcoef = gout @ cache["basis"]                  # (B, k)
    gbasis = gout.T @ cache["coef"]                # (P, k)
    # branch
    g["W3"] = cache["a2"].T @ gcoef
    g["b3"] = gcoef.sum(axis=0)
    gz2 = (gcoef @ q["W3"].T) * (cache["z2"] > 0)
    g["W2"] = cache["a1"].T @ gz2
    g["b2"] = gz2.sum(axis=0)
    gz1 = (gz2 @ q["W2"].T) * (cache["z1"] > 0)
    g["W1"] = cache["u"].T @ gz1
    g["b1"] = gz1.sum(axis=0)
    # trunk
    g["V3"] = cache["g2"].T @ gbasis
    g["c3"] = gbasis.sum(axis=0)
    gt2 = (gbasis @ q["V3"].T) * (cache["t2"] > 0)
    g["V2"] = cache["g1"].T @ gt2
    g["c2"] = gt2.sum(axis=0)
    gt1 = (gt2 @ q["V2"].T) * (cache["t1"] > 0)
    g["V1"] = cache["y"].T @ gt1
    g["c1"] = gt1.sum(axis=0)
    if parts is not None:
        parts.update(gz1=gz1, gz2=gz2, gt1=gt1, gt2=gt2, gcoef=gcoef, gbasis=gbasis)
    return pack(g, L)
