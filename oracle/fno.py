"""FP64 Fourier neural operator: forward, hand-derived backward, MSE, Adam.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Architecture (arXiv 2509.01416 section 4.2 and Appendix A1, carried to 2-D):
the input field and its grid coordinates are lifted pointwise to `width`
channels; `layers` Fourier layers follow, each the sum of a spectral path
(forward FFT, a complex linear map on the retained low modes, inverse FFT) and
a pointwise linear path, then an activation (none after the last layer); a
pointwise projection width -> 128 -> 1 returns the field.  The paper's 1-D
model has 549,569 parameters with width 64 and 16 modes (Table A1): that count
is the layout fc0 (2->64), four layers of (64x64x16 complex spectral weights,
64x64 pointwise + bias), fc1 (64->128), fc2 (128->1).  The 2-D model keeps
that layout with width 32, a 12 x 12 mode window and GELU.

2-D mode window on an (n, n) grid, rfft along x (the contiguous axis):
  kx in [0, modes), ky in [0, modes) (block 0) and ky in [n - modes, n)
  (block 1, the negative frequencies).

Flat parameter vector (float64 here), in this order:
  W0[3][w], b0[w];
  per layer: R[2][modes][modes][w_in][w_out][2] (re, im), W[w_in][w_out], b[w];
  P1[w][128], c1[128], P2[128], c2[1].
"""
from __future__ import annotations

from dataclasses import dataclass
from math import erf, sqrt

import numpy as np
from scipy.special import erf as _erf

PROJ = 128


@dataclass(frozen=True)
class Layout:
    width: int = 32
    modes: int = 12
    layers: int = 4
    in_ch: int = 3

    def offsets(self):
        w, m = self.width, self.modes
        off = {}
        o = 0

        def take(name, size):
            nonlocal o
            off[name] = (o, size)
            o += size
        take("W0", self.in_ch * w)
        take("b0", w)
        for l in range(self.layers):
            take(f"R{l}", 2 * m * m * w * w * 2)
            take(f"W{l + 1}", w * w)
            take(f"b{l + 1}", w)
        take("P1", w * PROJ)
        take("c1", PROJ)
        take("P2", PROJ)
        take("c2", 1)
        off["_total"] = (o, 0)
        return off

    @property
    def n_params(self) -> int:
        return self.offsets()["_total"][0]


def layout_param_count_1d(width: int, modes: int, layers: int) -> int:
    """Parameter count of the paper's 1-D FNO layout (Table A1 reading)."""
    lift = 2 * width + width
    per = modes * width * width * 2 + width * width + width
    proj = width * PROJ + PROJ + PROJ + 1
    return lift + layers * per + proj


def unpack(p: np.ndarray, L: Layout) -> dict:
    w, m = L.width, L.modes
    out = {}
    for name, (o, s) in L.offsets().items():
        if name == "_total":
            continue
        v = p[o:o + s]
        if name == "W0":
            v = v.reshape(L.in_ch, w)
        elif name.startswith("R"):
            v = v.reshape(2, m, m, w, w, 2)
            v = v[..., 0] + 1j * v[..., 1]
        elif name.startswith("W"):
            v = v.reshape(w, w)
        elif name == "P1":
            v = v.reshape(w, PROJ)
        out[name] = v
    return out


def pack(d: dict, L: Layout) -> np.ndarray:
    p = np.zeros(L.n_params)
    for name, (o, s) in L.offsets().items():
        if name == "_total":
            continue
        v = d[name]
        if name.startswith("R"):
            v = np.stack([v.real, v.imag], axis=-1)
        p[o:o + s] = np.asarray(v, dtype=np.float64).reshape(-1)
    return p


def init_params(L: Layout, seed: int) -> np.ndarray:
    """Seeded initialisation: linear layers U(-1/sqrt(fan_in), +), spectral
    weights (1/(w*w)) * U[0,1) for both real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w, m = L.width, L.modes
    d = {}

    def lin(fi, fo):
        k = 1.0 / np.sqrt(fi)
        return rng.uniform(-k, k, size=(fi, fo)), rng.uniform(-k, k, size=fo)
    d["W0"], d["b0"] = lin(L.in_ch, w)
    for l in range(L.layers):
        s = 1.0 / (w * w)
        d[f"R{l}"] = s * (rng.uniform(size=(2, m, m, w, w))
                          + 1j * rng.uniform(size=(2, m, m, w, w)))
        d[f"W{l + 1}"], d[f"b{l + 1}"] = lin(w, w)
    d["P1"], d["c1"] = lin(w, PROJ)
    P2, c2 = lin(PROJ, 1)
    d["P2"], d["c2"] = P2.reshape(PROJ), c2
    return pack(d, L)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def coords(n: int) -> tuple:
    """Cell-centre coordinates scaled to [0, 1]: (x/lx, y/ly) on (n, n)."""
    c = (np.arange(n) + 0.5) / n
    return np.broadcast_to(c[None, :], (n, n)), np.broadcast_to(c[:, None], (n, n))


def make_input(field: np.ndarray) -> np.ndarray:
    """(B, n, n) field -> (B, n, n, 3) network input (field, x, y)."""
    B, n, _ = field.shape
    xs, ys = coords(n)
    a = np.empty((B, n, n, 3))
    a[..., 0] = field
    a[..., 1] = xs
    a[..., 2] = ys
    return a


def _spectral(v, R, m):
    """Retained-mode spectral map of (B, n, n, w) -> (B, n, n, w)."""
    B, n, _, w = v.shape
    V = np.fft.rfft2(v, axes=(1, 2))                     # (B, n, n//2+1, w)
    Y = np.zeros_like(V)
    Y[:, :m, :m, :] = np.einsum("bykI,ykIO->bykO", V[:, :m, :m, :], R[0])
    Y[:, n - m:, :m, :] = np.einsum("bykI,ykIO->bykO", V[:, n - m:, :m, :], R[1])
    return np.fft.irfft2(Y, s=(n, n), axes=(1, 2)), V


def forward(p: np.ndarray, a: np.ndarray, L: Layout = Layout()):
    """a: (B, n, n, in_ch) -> (out (B, n, n), cache)."""
    P = unpack(p, L)
    m = L.modes
    v = a @ P["W0"] + P["b0"]
    cache = {"a": a, "v": [v], "z": [], "V": []}
    for l in range(L.layers):
        u, V = _spectral(v, P[f"R{l}"], m)
        z = u + v @ P[f"W{l + 1}"] + P[f"b{l + 1}"]
        cache["z"].append(z)
        cache["V"].append(V)
        v = gelu(z) if l < L.layers - 1 else z
        cache["v"].append(v)
    h = v @ P["P1"] + P["c1"]
    cache["h"] = h
    g = gelu(h)
    cache["g"] = g
    out = g @ P["P2"] + P["c2"][0]
    return out, cache


def backward(p: np.ndarray, cache: dict, gout: np.ndarray,
             L: Layout = Layout()):
    """Gradient of sum(gout * out) with respect to the parameters and input."""
    P = unpack(p, L)
    m = L.modes
    G = {k: np.zeros_like(v) for k, v in P.items()}
    B, n, _ = gout.shape
    g = cache["g"]
    G["P2"] = np.einsum("byxk,byx->k", g, gout)
    G["c2"] = np.array([gout.sum()])
    gg = gout[..., None] * P["P2"][None, None, None, :]
    gh = gg * gelu_grad(cache["h"])
    v = cache["v"][-1]
    G["P1"] = np.einsum("byxi,byxo->io", v, gh)
    G["c1"] = gh.sum(axis=(0, 1, 2))
    gv = gh @ P["P1"].T
    ckx = np.full(m, 2.0)
    ckx[0] = 1.0
    for l in reversed(range(L.layers)):
        z = cache["z"][l]
        gz = gv * gelu_grad(z) if l < L.layers - 1 else gv
        vin = cache["v"][l]
        G[f"W{l + 1}"] = np.einsum("byxi,byxo->io", vin, gz)
        G[f"b{l + 1}"] = gz.sum(axis=(0, 1, 2))
        gvin = gz @ P[f"W{l + 1}"].T
        # spectral path: u = irfft2(Y); gY = (c_kx / n^2) * rfft2(gz) on kept modes
        GZ = np.fft.rfft2(gz, axes=(1, 2))
        V = cache["V"][l]
        R = P[f"R{l}"]
        gR = np.zeros_like(R)
        gV = np.zeros_like(V)
        for blk, ys in ((0, slice(0, m)), (1, slice(n - m, n))):
            gY = GZ[:, ys, :m, :] * (ckx[None, None, :, None] / (n * n))
            gR[blk] = np.einsum("bykI,bykO->ykIO", np.conj(V[:, ys, :m, :]), gY)
            gV[:, ys, :m, :] = np.einsum("bykO,ykIO->bykI", gY, np.conj(R[blk]))
        G[f"R{l}"] = gR
        # forward V = rfft2(v) on kept modes: dL/dv = Re(sum_k gV e^{+i theta})
        # = n^2 * Re(ifft2 over the full grid of gV zero-padded)
        full = np.zeros((B, n, n, L.width), dtype=complex)
        full[:, :, : n // 2 + 1, :] = gV
        gvin = gvin + np.real(np.fft.ifft2(full, axes=(1, 2))) * (n * n)
        gv = gvin
    a = cache["a"]
    G["W0"] = np.einsum("byxi,byxo->io", a, gv)
    G["b0"] = gv.sum(axis=(0, 1, 2))
    ga = gv @ P["W0"].T
    return pack(G, L), ga


def mse(pred: np.ndarray, target: np.ndarray):
    """Mean squared error and its gradient with respect to pred."""
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, bias-corrected), in place; t >= 1."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return p


def gelu_scalar(z: float) -> float:
    return 0.5 * z * (1.0 + erf(z / sqrt(2.0)))
