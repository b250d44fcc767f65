"""Pins of the FP64 operator-network oracle: parameter counts, a brute-force
DFT of the spectral path, finite-difference gradients and hand-computed Adam
steps."""
import numpy as np
import pytest

from oracle import fno as F


def test_param_count_paper_1d_layout():
    # Table A1: FNO with 4 Fourier layers, 16 modes, width 64 -> 549,569
    assert F.layout_param_count_1d(64, 16, 4) == 549569


def test_param_count_2d_layout():
    assert F.Layout(width=32, modes=12, layers=4).n_params == 2368001


def _brute_spectral(v, R, m):
    """Direct double sum over the grid, no FFT library."""
    B, n, _, w = v.shape
    y = np.arange(n)
    u = np.zeros_like(v)
    kys = list(range(m)) + list(range(n - m, n))
    for b in range(B):
        for blk in (0, 1):
            for kyi in range(m):
                ky = kys[blk * m + kyi]
                for kx in range(m):
                    ph = np.exp(-2j * np.pi * (ky * y[:, None] + kx * y[None, :]) / n)
                    Vk = np.einsum("yxi,yx->i", v[b], ph)
                    Yk = Vk @ R[blk][kyi, kx]
                    ckx = 1.0 if kx == 0 else 2.0
                    basis = np.conj(ph)   # e^{+i theta}
                    u[b] += ckx / (n * n) * np.real(Yk[None, None, :] * basis[:, :, None])
    return u


def test_spectral_path_matches_brute_force_dft():
    rng = np.random.Generator(np.random.PCG64(1))
    B, n, w, m = 2, 8, 3, 3
    v = rng.standard_normal((B, n, n, w))
    R = rng.standard_normal((2, m, m, w, w)) + 1j * rng.standard_normal((2, m, m, w, w))
    u, _ = F._spectral(v, R, m)
    ref = _brute_spectral(v, R, m)
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()


def _loss(p, a, gout, L):
    out, _ = F.forward(p, a, L)
    return float(np.sum(out * gout))


def test_backward_matches_finite_differences():
    L = F.Layout(width=4, modes=3, layers=4)
    rng = np.random.Generator(np.random.PCG64(3))
    n, B = 12, 2
    p = F.init_params(L, seed=5)
    # larger spectral weights so that the spectral path matters in the check
    off = L.offsets()
    for l in range(L.layers):
        o, s = off[f"R{l}"]
        p[o:o + s] = rng.standard_normal(s) * 0.3
    a = F.make_input(rng.standard_normal((B, n, n)))
    gout = rng.standard_normal((B, n, n))
    out, cache = F.forward(p, a, L)
    gp, ga = F.backward(p, cache, gout, L)
    h = 1e-6
    idx = rng.choice(L.n_params, size=60, replace=False)
    # make sure every parameter block is probed
    idx = np.unique(np.concatenate([idx, [o for (o, s) in off.values() if s > 0]]))
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (_loss(p + e, a, gout, L) - _loss(p - e, a, gout, L)) / (2 * h)
        assert abs(fd - gp[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gp[i])
    for k in range(5):
        j = tuple(rng.integers(0, s) for s in a.shape[:-1]) + (0,)
        e = np.zeros_like(a)
        e[j] = h
        fd = (_loss(p, a + e, gout, L) - _loss(p, a - e, gout, L)) / (2 * h)
        assert abs(fd - ga[j]) <= 1e-6 * max(1.0, abs(fd))


def test_mse_gradient():
    rng = np.random.Generator(np.random.PCG64(8))
    x = rng.standard_normal((2, 3, 3))
    t = rng.standard_normal((2, 3, 3))
    l, g = F.mse(x, t)
    assert abs(l - np.mean((x - t) ** 2)) < 1e-15
    h = 1e-7
    e = np.zeros_like(x)
    e[1, 2, 0] = h
    fd = (F.mse(x + e, t)[0] - F.mse(x - e, t)[0]) / (2 * h)
    assert abs(fd - g[1, 2, 0]) < 1e-8


def test_adam_hand_computed():
    p = np.array([1.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    g1 = np.array([0.5, -0.25])
    F.adam_step(p, g1, m, v, 1, lr=0.1)
    # step 1: m_hat = g, v_hat = g^2 -> p -= lr * g/(|g| + eps)
    assert np.allclose(p, [1.0 - 0.1 * 0.5 / (0.5 + 1e-8),
                           -2.0 + 0.1 * 0.25 / (0.25 + 1e-8)], rtol=0, atol=1e-15)
    g2 = np.array([-1.0, 0.0])
    F.adam_step(p, g2, m, v, 2, lr=0.1)
    m_exp = 0.9 * 0.1 * g1 + 0.1 * g2
    v_exp = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mh = m_exp / (1 - 0.81)
    vh = v_exp / (1 - 0.999 ** 2)
    p_exp = np.array([1.0 - 0.1 * 0.5 / (0.5 + 1e-8),
                      -2.0 + 0.1 * 0.25 / (0.25 + 1e-8)]) - 0.1 * mh / (np.sqrt(vh) + 1e-8)
    assert np.allclose(p, p_exp, rtol=0, atol=1e-14)
    assert np.allclose(m, m_exp) and np.allclose(v, v_exp)


def test_gelu_values():
    # GELU(x) = x Phi(x): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    assert abs(F.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(F.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert F.gelu(np.array(0.0)) == 0.0
