"""Pins of the FP64 DeepONet oracle (section 4.1 Eq. 11, Appendix A1).

  * the paper's 1-D layout, branch [100, 200, 200, 100] and trunk
    [1, 200, 200, 100], has 141,200 parameters (App. A1);
  * with ReLU on positive pre-activations (all weights and inputs positive)
    the network is the product of its affine maps, written out here layer by
    layer (the inner product of Eq. 11 included);
  * the hand-derived backward equals central finite differences;
  * the output is linear in the branch's last layer and bilinear in the
    two nets' last layers (a scaling check that catches a dropped factor)."""
import numpy as np

from oracle import deeponet as D


def test_paper_parameter_count():
    assert D.PAPER_1D.count() == 141_200
    assert D.Layout().count() == 4096 * 200 + 200 + 200 * 200 + 200 + 200 * 100 + 100 \
        + 2 * 200 + 200 + 200 * 200 + 200 + 200 * 100 + 100


def test_positive_network_is_affine_composition():
    L = D.Layout(sensors=6, coords=2, hidden=5, basis=3)
    rng = np.random.Generator(np.random.PCG64(1))
    p = rng.uniform(0.1, 1.0, L.count())
    u = rng.uniform(0.1, 1.0, (4, 6))
    y = rng.uniform(0.1, 1.0, (7, 2))
    out, _ = D.forward(p, u, y, L)
    q = D.unpack(p, L)
    b = ((u @ q["W1"] + q["b1"]) @ q["W2"] + q["b2"]) @ q["W3"] + q["b3"]
    t = ((y @ q["V1"] + q["c1"]) @ q["V2"] + q["c2"]) @ q["V3"] + q["c3"]
    want = np.array([[sum(b[i, k] * t[j, k] for k in range(3)) for j in range(7)]
                     for i in range(4)])
    assert np.abs(out - want).max() < 1e-12 * np.abs(want).max()


def test_backward_matches_finite_differences():
    L = D.Layout(sensors=9, coords=2, hidden=7, basis=4)
    rng = np.random.Generator(np.random.PCG64(2))
    p = D.init_params(L, 3)
    u = rng.normal(size=(3, 9))
    y = D.grid_coords(3)
    gout = rng.normal(size=(3, 9))
    out, cache = D.forward(p, u, y, L)
    g = D.backward(p, cache, gout, L)
    h = 1e-6
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fp = np.sum(gout * D.forward(p + e, u, y, L)[0])
        fm = np.sum(gout * D.forward(p - e, u, y, L)[0])
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_inner_product_is_bilinear_in_the_last_layers():
    L = D.Layout(sensors=5, coords=2, hidden=4, basis=3)
    p = D.init_params(L, 4)
    u = np.random.Generator(np.random.PCG64(5)).normal(size=(2, 5))
    y = D.grid_coords(2)
    q = D.unpack(p, L)
    out, _ = D.forward(p, u, y, L)
    q2 = dict(q, W3=2.0 * q["W3"], b3=2.0 * q["b3"], V3=3.0 * q["V3"], c3=3.0 * q["c3"])
    out2, _ = D.forward(D.pack(q2, L), u, y, L)
    assert np.abs(out2 - 6.0 * out).max() < 1e-12 * np.abs(out).max()


def test_grid_coords_are_cell_centres_x_fastest():
    c = D.grid_coords(4)
    assert c.shape == (16, 2)
    assert np.allclose(c[1], [0.375, 0.125]) and np.allclose(c[4], [0.125, 0.375])
