"""Seeded synthetic inputs for the fixed-source S_N workloads.

This module is the only code shared by the HIP path's callers (tests, bench) and
the FP64 oracle's callers.  It holds no arithmetic of the method itself: it only
draws inputs (quadrature sets, Gaussian-random-field sources, cross-section
fields) and names the workloads.  Nothing here sweeps, iterates or evaluates a
network.

Paper anchors (arXiv 2509.01416):
  * the problem data of the fixed-source transport equation -- total and
    isotropic scattering cross sections and an isotropic source -- follow
    section 5.1, Eq. 12;
  * sources are Gaussian random fields (Appendix A1); the paper's 1-D slab is
    10 cm long with 0.1 cm cells and uses S_N angular discretisation
    (section 5.1, the paragraph after Eq. 24);
  * the 2-D x-y analogues (domain 10 x 10 mfp, level-symmetric quadrature) are
    this library's extension of that 1-D setup (section 6 notes the recast is
    unchanged in higher dimension).

Conventions:
  * fields are float64 numpy arrays, shape (ny, nx), x fastest (cell-major);
  * quadrature weights sum to 1 over all directions (the paper's Gauss-Legendre
    weights sum to 2 with a 1/2 on the emission; both give the same scalar
    flux).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# --------------------------------------------------------------------------
# quadrature sets
# --------------------------------------------------------------------------

# First cosine of the level-symmetric LQ_N sets (Lewis & Miller, "Computational
# Methods of Neutron Transport", table of LQ_N quadratures).
LQ_MU1 = {2: 0.5773503, 4: 0.3500212, 6: 0.2666355, 8: 0.2182179,
          12: 0.1672126, 16: 0.1389568}


@dataclass(frozen=True)
class Quadrature:
    """A discrete-ordinates set.  mu (x-cosine), eta (y-cosine, None in 1-D), w.

    Weights sum to 1; the set is symmetric under mu -> -mu (and eta -> -eta).
    """
    mu: np.ndarray
    eta: Optional[np.ndarray]
    w: np.ndarray
    name: str = ""

    @property
    def n_dir(self) -> int:
        return int(self.w.shape[0])


def gauss_legendre(n: int) -> Quadrature:
    """1-D S_n Gauss-Legendre set, weights halved so they sum to 1."""
    mu, w = np.polynomial.legendre.leggauss(n)
    return Quadrature(mu=np.ascontiguousarray(mu), eta=None,
                      w=np.ascontiguousarray(w / 2.0), name=f"GL{n}")


def _sphere_moment(a: int, b: int, c: int) -> float:
    """(1/4pi) * integral over the unit sphere of x^a y^b z^c, a,b,c even."""
    return (2.0 * math.gamma((a + 1) / 2) * math.gamma((b + 1) / 2)
            * math.gamma((c + 1) / 2) / math.gamma((a + b + c + 3) / 2)
            / (4.0 * math.pi))


def level_symmetric_octant(n: int, mu1: Optional[float] = None):
    """Points and weights of one octant of the level-symmetric LQ_n set.

    Cosines: mu_i^2 = mu_1^2 + (i-1) * 2(1 - 3 mu_1^2)/(n-2), i = 1..n/2; the
    octant points are the triples (mu_i, mu_j, mu_k) with i + j + k = n/2 + 2.
    One weight per permutation class, fitted by least squares to the even
    moments <mu^a eta^b> (a + b <= n) of the octant.  Octant weights sum to 1.
    Returns (points (P,3), weights (P,), class labels).
    """
    if n < 4 or n % 2:
        raise ValueError("level-symmetric order must be even and >= 4")
    mu1 = LQ_MU1[n] if mu1 is None else mu1
    half = n // 2
    d = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (n - 2)
    cos = np.sqrt(mu1 * mu1 + np.arange(half) * d)
    pts, cls = [], []
    for i in range(1, half + 1):
        for j in range(1, half + 1):
            k = half + 2 - i - j
            if k >= 1:
                pts.append((cos[i - 1], cos[j - 1], cos[k - 1]))
                cls.append(tuple(sorted((i, j, k))))
    pts = np.array(pts)
    classes = sorted(set(cls))
    rows, rhs = [], []
    for a in range(0, n + 1, 2):
        for b in range(0, n + 1 - a, 2):
            rows.append([sum(pts[p, 0] ** a * pts[p, 1] ** b
                             for p in range(len(pts)) if cls[p] == c)
                         for c in classes])
            rhs.append(_sphere_moment(a, b, 0))
    cw, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
    w = np.array([cw[classes.index(c)] for c in cls])
    w = w / w.sum()          # the zeroth moment exactly (fit residual ~1e-9)
    return pts, w, cls


def level_symmetric_2d(n: int) -> Quadrature:
    """2-D x-y LQ_n set: n(n+2)/2 directions (40 for S8, 144 for S16).

    The upper-hemisphere octant points (mu, eta, xi>0) are placed in the four
    (sign mu, sign eta) quadrants; the xi<0 half is folded in, so each 2-D
    direction carries octant_weight/4 and all weights sum to 1.
    Order: quadrant-major (++, -+, --, +-), then octant point order.
    """
    pts, w, _ = level_symmetric_octant(n)
    mus, etas, ws = [], [], []
    for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        mus.append(sx * pts[:, 0])
        etas.append(sy * pts[:, 1])
        ws.append(w / 4.0)
    return Quadrature(mu=np.concatenate(mus), eta=np.concatenate(etas),
                      w=np.concatenate(ws), name=f"LQ{n}")


# --------------------------------------------------------------------------
# Gaussian random fields
# --------------------------------------------------------------------------

def grf_2d(n: int, length: float, seed: int, mean: float = 1.0,
           std: float = 0.3, scale: float = 1.0, clip_min: Optional[float] = 0.0
           ) -> np.ndarray:
    """Stationary Gaussian random field on an n x n cell-centred grid.

    Squared-exponential covariance exp(-r^2 / (2 l^2)), sampled by circulant
    embedding on a 2n x 2n periodic grid (negative eigenvalues clipped to 0).
    `length` is the physical side of the square; cell size = length / n.
    `scale` is the correlation length.  numpy PCG64 with the given seed.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = length / n
    m = 2 * n
    k = np.arange(m)
    d = np.minimum(k, m - k) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    cov = np.exp(-r2 / (2.0 * scale * scale))
    lam = np.maximum(np.real(np.fft.fft2(cov)), 0.0)
    xi = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    f = np.fft.fft2(np.sqrt(lam / (m * m)) * xi)
    g = mean + std * np.real(f)[:n, :n]
    if clip_min is not None:
        g = np.maximum(g, clip_min)
    return np.ascontiguousarray(g)


def grf_1d(n: int, length: float, seed: int, mean: float, std: float,
           scale: float, clip_min: Optional[float] = 0.0) -> np.ndarray:
    """1-D analogue of grf_2d (circulant embedding on a 2n periodic grid)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = length / n
    m = 2 * n
    k = np.arange(m)
    d = np.minimum(k, m - k) * h
    cov = np.exp(-d * d / (2.0 * scale * scale))
    lam = np.maximum(np.real(np.fft.fft(cov)), 0.0)
    xi = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    f = np.fft.fft(np.sqrt(lam / m) * xi)
    g = mean + std * np.real(f)[:n]
    if clip_min is not None:
        g = np.maximum(g, clip_min)
    return np.ascontiguousarray(g)


# --------------------------------------------------------------------------
# cross-section fields
# --------------------------------------------------------------------------

def cell_centres(n: int, length: float) -> np.ndarray:
    h = length / n
    return (np.arange(n) + 0.5) * h


def sinusoid_field(nx: int, ny: int, lx: float, ly: float, base: float,
                   amp: float, kind: str = "sin") -> np.ndarray:
    """base + amp * f(2 pi x / lx) f(2 pi y / ly) at cell centres, f = sin|cos."""
    x = cell_centres(nx, lx)
    y = cell_centres(ny, ly)
    f = np.sin if kind == "sin" else np.cos
    return base + amp * np.outer(f(2 * np.pi * y / ly), f(2 * np.pi * x / lx))


def random_line_mask(nx: int, ny: int, lx: float, ly: float, seed: int
                     ) -> np.ndarray:
    """Boolean (ny, nx) mask: True on one side of a seeded random line.

    Angle ~ U[0, 2 pi), point ~ U[0.25 L, 0.75 L]^2; the side of each cell
    centre decides its region.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.0, 2.0 * np.pi)
    x0 = rng.uniform(0.25 * lx, 0.75 * lx)
    y0 = rng.uniform(0.25 * ly, 0.75 * ly)
    x = cell_centres(nx, lx)[None, :]
    y = cell_centres(ny, ly)[:, None]
    return ((x - x0) * np.cos(theta) + (y - y0) * np.sin(theta)) < 0.0


def block_field(nx: int, ny: int, nb: int, lo: float, hi: float,
                rng: np.random.Generator) -> np.ndarray:
    """Piecewise-constant field on an nb x nb block layout, values U[lo, hi]."""
    vals = rng.uniform(lo, hi, size=(nb, nb))
    bi = (np.arange(ny) * nb) // ny
    bj = (np.arange(nx) * nb) // nx
    return np.ascontiguousarray(vals[bi][:, bj])


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

BC_VACUUM = 0
BC_REFLECTIVE = 1


@dataclass
class Instance:
    """One fixed-source problem: sigma_t, sigma_s, source on a uniform grid;
    sigma_s1 (optional) is the first Legendre moment of scattering."""
    nx: int
    ny: int
    lx: float
    ly: float
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    source: np.ndarray
    bc: Tuple[int, int, int, int] = (0, 0, 0, 0)   # x-, x+, y-, y+
    dim: int = 2
    sigma_s1: Optional[np.ndarray] = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    quad: Quadrature
    tol: float
    description: str = ""
    extra: dict = field(default_factory=dict)

    def cell_angles(self) -> int:
        """Cell-angle updates in one sweep of every instance."""
        return sum(i.cells for i in self.instances) * self.quad.n_dir


def slab_1d() -> Workload:
    """1-D slab, 200 cells on [0, 10] mfp, S8 Gauss-Legendre, sigma_t = 1,
    c = 0.9, uniform q = 1, vacuum; FP64 oracle acceptance case
    (tolerance 1e-8 on the max relative scalar-flux change)."""
    n = 200
    inst = Instance(nx=n, ny=1, lx=10.0, ly=1.0,
                    sigma_t=np.ones((1, n)), sigma_s=np.full((1, n), 0.9),
                    source=np.ones((1, n)), dim=1)
    return Workload("slab1d_200_S8", [inst], gauss_legendre(8), tol=1e-8,
                    description="1-D slab 200 cells S8 GL c=0.9 q=1 vacuum")


def sinusoid_128(n: int = 128) -> Workload:
    """Single 2-D instance: 128^2 on 10x10 mfp, LQ S8,
    sigma_t = 1 + 0.5 sin sin, c = 0.9, GRF source (seed 2), vacuum."""
    st = sinusoid_field(n, n, 10.0, 10.0, 1.0, 0.5)
    q = grf_2d(n, 10.0, seed=2)
    inst = Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st,
                    sigma_s=0.9 * st, source=q)
    return Workload(f"sinusoid_{n}_S8", [inst], level_symmetric_2d(8),
                    tol=1e-6, description="128^2 S8 sinusoidal sigma_t c=0.9")


def batched_uneven(count: int = 256, sizes=(32, 48, 64, 96, 128)) -> Workload:
    """`count` uneven 2-D instances (seed 3000+i): side ~ U{sizes},
    4x4-block sigma_t ~ U[0.5, 2], c ~ U[0.5, 0.95], GRF source; LQ S8."""
    insts = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(3000 + i))
        n = int(rng.choice(np.array(sizes)))
        st = block_field(n, n, 4, 0.5, 2.0, rng)
        c = rng.uniform(0.5, 0.95)
        q = grf_2d(n, 10.0, seed=int(rng.integers(1 << 31)))
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st,
                              sigma_s=c * st, source=q))
    return Workload(f"batched_uneven_{count}_S8", insts, level_symmetric_2d(8),
                    tol=1e-6, description="uneven batched S8 solves")


SIGMA_T_STAR = 1.0
SIGMA_S_STAR = 0.8


def fno_training_set(count: int = 2000, n: int = 64, seed0: int = 40000
                     ) -> Workload:
    """Training sources for the operator network: constant sigma_t = 1,
    c = 0.8 (the single training configuration p*), GRF sources."""
    insts = []
    st = np.full((n, n), SIGMA_T_STAR)
    ss = np.full((n, n), SIGMA_S_STAR)
    for j in range(count):
        q = grf_2d(n, 10.0, seed=seed0 + j)
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st,
                              sigma_s=ss, source=q))
    return Workload(f"fno_train_{count}_{n}", insts, level_symmetric_2d(8),
                    tol=1e-7, description="training set at p*")


def fno_eval_set(family: str, count: int = 64, n: int = 64,
                 seed0: int = 41000) -> Workload:
    """Evaluation instances for the recast warm start.

    family 'sinusoid': sigma_t = 1 + 0.3 sin sin, c = 0.8 + 0.1 cos cos;
    family 'line': random-line split, (sigma_t, c) = (0.7, 0.85) | (1.3, 0.75);
    family 'fallback': random-line split, sigma_a up to 0.6 (> 2 sigma_a*).
    """
    insts = []
    for j in range(count):
        seed = seed0 + j
        q = grf_2d(n, 10.0, seed=seed)
        if family == "sinusoid":
            st = sinusoid_field(n, n, 10.0, 10.0, 1.0, 0.3, "sin")
            c = sinusoid_field(n, n, 10.0, 10.0, 0.8, 0.1, "cos")
        elif family == "line":
            m = random_line_mask(n, n, 10.0, 10.0, seed + 500)
            st = np.where(m, 0.7, 1.3)
            c = np.where(m, 0.85, 0.75)
        elif family == "fallback":
            m = random_line_mask(n, n, 10.0, 10.0, seed + 500)
            st = np.where(m, 1.0, 1.5)
            c = np.where(m, 0.8, 0.6)
        else:
            raise ValueError(family)
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st,
                              sigma_s=c * st, source=q))
    return Workload(f"fno_eval_{family}_{count}_{n}", insts,
                    level_symmetric_2d(8), tol=1e-6)


def paper_slab_p1(case: int, seed: int = 43000) -> Workload:
    """The paper's 1-D fixed-source setting with linearly anisotropic
    scattering (section 5.1, Eq. 25): 100 cells over 10 cm, S32
    Gauss-Legendre, vacuum faces, sigma_s1 = 0.3, a GRF source (mean 0.07,
    variance 3e-4, correlation length 1.2 cm).  case 2: sigma_t = 1.2,
    sigma_s0 = 0.8; case 3: sinusoidal sigma_t and sigma_s0 (the paper gives
    their shapes only in a figure; sigma_t = 1 + 0.2 sin(2 pi x / 5),
    sigma_s0 = 0.6 + 0.15 sin(2 pi x / 5) stand in)."""
    n, L = 100, 10.0
    x = cell_centres(n, L)
    if case == 2:
        st, ss = np.full(n, 1.2), np.full(n, 0.8)
    elif case == 3:
        st = 1.0 + 0.2 * np.sin(2 * np.pi * x / 5.0)
        ss = 0.6 + 0.15 * np.sin(2 * np.pi * x / 5.0)
    else:
        raise ValueError(case)
    q = grf_1d(n, L, seed=seed + case, mean=0.07, std=3e-4 ** 0.5, scale=1.2)
    inst = Instance(nx=n, ny=1, lx=L, ly=1.0, sigma_t=st.reshape(1, n),
                    sigma_s=ss.reshape(1, n), source=q.reshape(1, n), dim=1,
                    sigma_s1=np.full((1, n), 0.3))
    return Workload(f"paper_slab_case{case}_p1", [inst], gauss_legendre(32), tol=1e-6,
                    description="1-D slab with P1 scattering")


def p1_eval_set(count: int = 8, n: int = 64, seed0: int = 42000) -> Workload:
    """x-y analogue of the paper's Case 2 on the network grid: sigma_t = 1.1,
    sigma_s0 = 0.85 (sigma_a = 0.25, inside the recast's convergence range
    around sigma_a* = 0.2), sigma_s1 = 0.3, a GRF source per instance,
    10 x 10 mfp, vacuum faces, S8."""
    insts = []
    for j in range(count):
        q = grf_2d(n, 10.0, seed=seed0 + j)
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=np.full((n, n), 1.1),
                              sigma_s=np.full((n, n), 0.85), source=q,
                              sigma_s1=np.full((n, n), 0.3)))
    return Workload(f"p1_eval_{count}_{n}", insts, level_symmetric_2d(8), tol=1e-6,
                    description="Case 2 analogue with P1 scattering")


def hard_two_region(count: int = 16, n: int = 256) -> Workload:
    """`count` instances of n^2 cells, LQ S16, sigma_t in {1, 5} split by a
    seeded random line (seed 5000+i), c = 0.99, GRF source, vacuum."""
    insts = []
    for i in range(count):
        m = random_line_mask(n, n, 10.0, 10.0, 5000 + i)
        st = np.where(m, 1.0, 5.0)
        q = grf_2d(n, 10.0, seed=5500 + i)
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st,
                              sigma_s=0.99 * st, source=q))
    return Workload(f"two_region_{count}x{n}_S16", insts, level_symmetric_2d(16),
                    tol=1e-6, description="c=0.99 two-region S16")


def random_instance(nx: int, ny: int, seed: int, lx: float = 10.0,
                    ly: float = 10.0, c_range=(0.3, 0.9), st_range=(0.5, 2.0),
                    bc=(0, 0, 0, 0)) -> Instance:
    """Small heterogeneous instance for parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = rng.uniform(*st_range, size=(ny, nx))
    c = rng.uniform(*c_range, size=(ny, nx))
    q = rng.uniform(0.0, 2.0, size=(ny, nx))
    return Instance(nx=nx, ny=ny, lx=lx, ly=ly, sigma_t=st, sigma_s=c * st,
                    source=q, bc=tuple(bc))


def eigen_case1_2d(count: int = 16, n: int = 256, quad_order: int = 16) -> Workload:
    """k-eigenvalue workload, the x-y analogue of eigen Case 1 (section 5.2):
    sigma_t = 1, sigma_s = 0.5, nu_sigma_f = 0.9 (sigma_f = 0.3 with the
    reading nu = 3) on a 10 x 10 mfp square, vacuum faces, n^2 cells,
    level-symmetric S_N.  Instance i carries a seeded +-2 % GRF perturbation
    of nu_sigma_f (seed 7000+i) so the batch holds distinct problems.
    extra["nu_sigma_f"] lists the fission fields; the sources are zero."""
    insts, nsf = [], []
    for i in range(count):
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=np.full((n, n), 1.0),
                              sigma_s=np.full((n, n), 0.5), source=np.zeros((n, n))))
        g = grf_2d(n, 10.0, seed=7000 + i)
        nsf.append(0.9 * (1.0 + 0.02 * (g - g.mean()) / max(g.std(), 1e-12)))
    return Workload(f"eigen_case1_{count}x{n}_S{quad_order}", insts,
                    level_symmetric_2d(quad_order), tol=1e-4,
                    description="2-D eigen Case 1 analogue", extra={"nu_sigma_f": nsf})


def eigen_sine_64(count: int = 16) -> Workload:
    """k-eigenvalue workload on the network's 64 x 64 grid (10 x 10 mfp,
    vacuum, S8): sinusoidal sigma_t, sigma_s and nu_sigma_f in the manner of
    eigen Case 2 (section 5.2), whose exact forms the paper does not print;
    instance i shifts the phases by a seeded offset (seed 7500+i)."""
    n = 64
    x = (np.arange(n) + 0.5) * 10.0 / n
    X, Y = np.meshgrid(x, x)
    insts, nsf = [], []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(7500 + i))
        a, b = rng.uniform(0.0, 10.0, 2)
        st = 1.0 + 0.3 * np.sin(2 * np.pi * (X + a) / 10.0) * np.cos(2 * np.pi * (Y + b) / 10.0)
        ss = st * (0.75 + 0.1 * np.sin(2 * np.pi * (X + Y + a) / 10.0))
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=st, sigma_s=ss,
                              source=np.zeros((n, n))))
        nsf.append(0.25 + 0.1 * np.cos(2 * np.pi * (X + b) / 5.0))
    return Workload(f"eigen_sine_{count}x64_S8", insts, level_symmetric_2d(8), tol=1e-4,
                    description="2-D sinusoidal eigen problems on the network grid",
                    extra={"nu_sigma_f": nsf})


# Tables 8-9 (section 5.3): sigma_s^{g->h} (rows g, columns h), nu,
# sigma_t, sigma_f, chi of the three-group problem.
THREE_GROUP_SS = ((0.024, 0.171, 0.033), (0.0, 0.600, 0.275), (0.0, 0.0, 2.000))
THREE_GROUP_NU = (3.0, 2.5, 2.0)
THREE_GROUP_ST = (0.240, 0.975, 3.000)
THREE_GROUP_SF = (0.006, 0.060, 0.900)
THREE_GROUP_CHI = (0.96, 0.04, 0.0)


def three_group_2d(count: int = 16, n: int = 256, quad_order: int = 16) -> Workload:
    """x-y analogue of the three-group problem (section 5.3, Tables 8-9) on
    a 10 x 10 cm square, vacuum faces, n^2 cells, level-symmetric S_N.
    Instance i scales every cross section of group g by a seeded +-2 % GRF
    field (seed 8000 + 3i + g), so the batch holds distinct problems.
    extra["groups"][i] = dict(sigma_t, sigma_s (3 x 3, None = zero),
    nu_sigma_f, chi) as numpy fields."""
    insts, groups = [], []
    for i in range(count):
        sc = []
        for g in range(3):
            f = grf_2d(n, 10.0, seed=8000 + 3 * i + g)
            sc.append(1.0 + 0.02 * (f - f.mean()) / max(f.std(), 1e-12))
        groups.append(dict(
            sigma_t=[THREE_GROUP_ST[g] * sc[g] for g in range(3)],
            sigma_s=[[THREE_GROUP_SS[g][h] * sc[g] if (h >= g and THREE_GROUP_SS[g][h] != 0.0)
                      else None for h in range(3)] for g in range(3)],
            nu_sigma_f=[THREE_GROUP_NU[g] * THREE_GROUP_SF[g] * sc[g] for g in range(3)],
            chi=list(THREE_GROUP_CHI)))
        insts.append(Instance(nx=n, ny=n, lx=10.0, ly=10.0, sigma_t=sc[0], sigma_s=np.zeros((n, n)),
                              source=np.zeros((n, n))))
    return Workload(f"three_group_{count}x{n}_S{quad_order}", insts,
                    level_symmetric_2d(quad_order), tol=1e-4,
                    description="2-D three-group eigen problems (Tables 8-9)",
                    extra={"groups": groups})
