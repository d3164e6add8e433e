"""Seeded synthetic inputs for the tests and the benchmark.

Holds no arithmetic of the DG method: only problem parameters, coefficient
fields, manufactured solutions and random vectors.  Both the HIP path and
the CPU oracle receive the same inputs from here.

Workloads (the paper's public SPE10 data set is not available, so W3 is a
synthetic stand-in with SPE10's shape and contrast):
  W1  Poisson, unit cube, 8^3 cells, p=2, sigma = 2p(p+1) = 12, K = I,
      homogeneous Dirichlet, f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z).
  W2  Poisson, unit cube, 32^3 cells, p=4, K = I, u = seeded random
      polynomial of total degree 3 (seed 2), g = u, f = -lap u.
  W3  60 x 220 x 85 cells of 20 x 10 x 2 (ft), p=2, per-cell diagonal K:
      log10 Kx = per z-layer Gaussian-filtered N(0,1) noise (sigma 5 cells,
      reflecting), standardised per layer, times 1.5, clipped to [-3, 3];
      Ky = Kx, Kz = 0.1 Kx (seed 3); Neumann on z faces, Dirichlet 0 on the
      lateral faces; f = +1 in the cell column (0, 0, :) and -1 in
      (59, 219, :).
  W4  unit cube, 48^3 cells, p=3, K = 1e-3 I, b = (-(y-1/2), x-1/2, 0.2),
      c = 0, f = 1, homogeneous Dirichlet.
  Pe2000  the paper's convection-dominated problem (Sec. 4.3): [0,1]^2 x
      [0,2], b = (1,0,0) or (1, 0.5, 0.3), kappa = max b_i h / 2000,
      u = X(1-X) Y(1-Y) Z(1-Z), homogeneous Dirichlet.
  Inhom  second diffusion test (Sec. 4.2): [0,1]^2 x [0,2], axis-aligned
      K(x) = diag(P_1(x), P_2(y), P_3(z)), P_k = p0_k + p2_k s^2,
      c = 1e-8 |x|^2, Gaussian f, g (Dirichlet) and j (Neumann on x = 1).
  W5  serving mix: N in {8,12,16,24,32} cells per side, p in {2,3,4}, K_T =
      exp(Z_T) I with Z ~ N(0,1), random load vector (seed 5000 + i),
      homogeneous Dirichlet.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PI = np.pi


@dataclass
class Workload:
    name: str
    cells: tuple
    lengths: tuple
    p: int
    bc: tuple
    sigma: float | None
    K: object
    c: object = 0.0
    b0: tuple = (0.0, 0.0, 0.0)
    B: tuple = ((0.0,) * 3,) * 3
    f: object = None      # callable (npts,3) -> (npts,) or None
    g: object = None      # Dirichlet data
    j: object = None      # Neumann data
    exact: object = None  # exact solution, when known
    info: dict = field(default_factory=dict)
    coarse: str = "auto"  # coarse space of the V-cycle: "auto" (Q1 if b = 0, else P0), "q1" or "p0"
    # axis-quadratic coefficient field: kfield = (q0, q1, q2) (3 each),
    # K_kk(x) = q0_k + q1_k x_k + q2_k x_k^2; cfield = (c0, c2), c = c0 + c2 |x|^2
    kfield: tuple | None = None
    cfield: tuple = (0.0, 0.0)
    nrot: tuple | None = None  # orthonormal rows n_m: K(x) = sum_m P_m(x_m) n_m n_m^T (None: n_m = e_m)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.cells))

    @property
    def ndof(self) -> int:
        return self.ncell * (self.p + 1) ** 3


def _sinsin(x):
    return np.sin(PI * x[:, 0]) * np.sin(PI * x[:, 1]) * np.sin(PI * x[:, 2])


def w1(cells=(8, 8, 8)) -> Workload:
    return Workload("poisson-8^3-p2", cells, (1.0, 1.0, 1.0), 2, ("D",) * 6, 12.0, 1.0,
                    f=lambda x: 3 * PI**2 * _sinsin(x), exact=_sinsin)


def random_poly3(seed: int = 2):
    """u = sum_{a+b+c <= 3} C_abc x^a y^b z^c, C ~ N(0,1); returns (u, -lap u)."""
    rng = np.random.default_rng(seed)
    exps = [(a, b, c) for a in range(4) for b in range(4) for c in range(4) if a + b + c <= 3]
    C = rng.normal(size=len(exps))

    def u(x):
        out = np.zeros(len(x))
        for (a, b, c), m in zip(exps, C):
            out += m * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
        return out

    def mlap(x):
        out = np.zeros(len(x))
        for (a, b, c), m in zip(exps, C):
            if a > 1:
                out -= m * a * (a - 1) * x[:, 0] ** (a - 2) * x[:, 1] ** b * x[:, 2] ** c
            if b > 1:
                out -= m * b * (b - 1) * x[:, 0] ** a * x[:, 1] ** (b - 2) * x[:, 2] ** c
            if c > 1:
                out -= m * c * (c - 1) * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 2)
        return out

    return u, mlap


def w2(cells=(32, 32, 32), p=4) -> Workload:
    u, mlap = random_poly3(2)
    return Workload("poisson-32^3-p4", cells, (1.0, 1.0, 1.0), p, ("D",) * 6, None, 1.0, f=mlap, g=u, exact=u)


def spe10_like_K(cells=(60, 220, 85), seed: int = 3) -> np.ndarray:
    """Layered log-normal diagonal permeability, shape (ncell, 3)."""
    from scipy.ndimage import gaussian_filter

    nx, ny, nz = cells
    rng = np.random.default_rng(seed)
    logk = np.empty((nz, ny, nx))
    for k in range(nz):
        layer = gaussian_filter(rng.normal(size=(ny, nx)), sigma=5.0, mode="reflect")
        layer = (layer - layer.mean()) / layer.std()
        logk[k] = np.clip(1.5 * layer, -3.0, 3.0)
    kx = 10.0 ** logk.reshape(-1)  # x fastest, then y, then z
    return np.stack([kx, kx, 0.1 * kx], axis=1)


def w3(cells=(60, 220, 85)) -> Workload:
    nx, ny, nz = cells
    lengths = (20.0 * nx, 10.0 * ny, 2.0 * nz)
    hx, hy = lengths[0] / nx, lengths[1] / ny

    def f(x):
        out = np.zeros(len(x))
        out[(x[:, 0] < hx) & (x[:, 1] < hy)] = 1.0
        out[(x[:, 0] > lengths[0] - hx) & (x[:, 1] > lengths[1] - hy)] = -1.0
        return out

    return Workload("spe10-like-60x220x85-p2", cells, lengths, 2, ("D", "D", "D", "D", "N", "N"), None,
                    spe10_like_K(cells), f=f)


def w4(cells=(48, 48, 48), p=3) -> Workload:
    return Workload("convection-48^3-p3", cells, (1.0, 1.0, 1.0), p, ("D",) * 6, None, 1e-3,
                    b0=(0.5, -0.5, 0.2), B=((0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
                    f=lambda x: np.ones(len(x)))


def pe2000(b=(1.0, 0.0, 0.0), p=3, cells=None) -> Workload:
    """Convection-dominated problem of the paper's Sec. 4.3:
    -kappa lap u + div(b u) = f on [0,1] x [0,1] x [0,2], b constant, grid
    Peclet number max_i b_i h / kappa = 2000, exact solution
    u = X(1-X) Y(1-Y) Z(1-Z) with X = x/Lx, ..., zero on the boundary
    (homogeneous Dirichlet).  Default grids: the paper's isotropic grids
    per degree (p=2: 56x56x112, p=3: 32x32x64, p=4: 20x20x40)."""
    if cells is None:
        cells = {1: (128, 128, 256), 2: (56, 56, 112), 3: (32, 32, 64), 4: (20, 20, 40)}[p]
    lengths = (1.0, 1.0, 2.0)
    h = lengths[0] / cells[0]
    kappa = max(b) * h / 2000.0
    bx, by, bz = b

    def parts(x):
        X, Y, Z = x[:, 0] / lengths[0], x[:, 1] / lengths[1], x[:, 2] / lengths[2]
        return X * (1 - X), Y * (1 - Y), Z * (1 - Z), (1 - 2 * X) / lengths[0], (1 - 2 * Y) / lengths[1], \
            (1 - 2 * Z) / lengths[2]

    def u(x):
        qx, qy, qz, _, _, _ = parts(x)
        return qx * qy * qz

    def f(x):
        qx, qy, qz, dx, dy, dz = parts(x)
        lap = -2 * (qy * qz / lengths[0] ** 2 + qx * qz / lengths[1] ** 2 + qx * qy / lengths[2] ** 2)
        return -kappa * lap + bx * dx * qy * qz + by * qx * dy * qz + bz * qx * qy * dz

    name = "convection-pe2000-b%s-%dx%dx%d-p%d" % ("x" if b[1] == 0 and b[2] == 0 else "xyz", *cells, p)
    return Workload(name, tuple(cells), lengths, p, ("D",) * 6, None, kappa, b0=tuple(b), f=f, exact=u,
                    info={"kappa": kappa, "peclet": 2000.0})


def field_functions(kfield, cfield=(0.0, 0.0), nrot=None):
    """Callables K(x) and c(x) -> (npts,) of a quadratic coefficient field:
    K(x) -> (npts, 3) diagonal when nrot is None, else the full tensor
    sum_m P_m(x_m) n_m n_m^T -> (npts, 3, 3)."""
    q0, q1, q2 = (np.asarray(v, dtype=np.float64) for v in kfield)
    c0, c2 = (float(v) for v in cfield)
    cfun = lambda x: c0 + c2 * np.sum(x ** 2, axis=1)  # noqa: E731
    if nrot is None:
        return (lambda x: q0 + q1 * x + q2 * x ** 2), cfun
    n = np.asarray(nrot, dtype=np.float64)
    return (lambda x: np.einsum("qm,mk,ml->qkl", q0 + q1 * x + q2 * x ** 2, n, n)), cfun


def rotation(a: float, b: float, c: float) -> np.ndarray:
    """Orthonormal basis (rows) from three angles (z-y-x rotations)."""
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    Rz = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
    Ry = np.array([[cb, 0.0, sb], [0.0, 1.0, 0.0], [-sb, 0.0, cb]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, cc, -sc], [0.0, sc, cc]])
    return (Rz @ Ry @ Rx).T


def gaussian(x0, s: float = 0.1):
    x0 = np.asarray(x0, dtype=np.float64)
    return lambda x: np.exp(-np.sum((x - x0) ** 2, axis=1) / (2.0 * s * s))


def inhomogeneous(p=4, cells=None, kfield=((1.0, 0.5, 2.0), (0.0, 0.0, 0.0), (3.0, 1.0, 0.5)),
                  nrot=None) -> Workload:
    """Second diffusion test of Sec. 4.2: -div(K(x) grad u) + c(x) u = f on
    [0,1] x [0,1] x [0,2] with K(x) = sum_k P_k(x_k) n_k n_k^T, n_k = e_k,
    P_k(s) = p0_k + p2_k s^2 (the paper leaves p0, p2 open; here
    p0 = (1, 0.5, 2), p2 = (3, 1, 0.5)), c(x) = 1e-8 |x|^2; Neumann on the
    face x = 1 with j a Gaussian at (1, 0.5, 0.5), Dirichlet elsewhere with
    g a Gaussian at (0, 0.5, 0.5), f a Gaussian at (0.75, 0.5, 0.3), all of
    width 0.1.  Default grid: the paper's isotropic grid for degree p."""
    if cells is None:
        cells = {1: (128, 128, 256), 2: (56, 56, 112), 3: (32, 32, 64), 4: (20, 20, 40)}[p]
    name = "inhomogeneous%s-%dx%dx%d-p%d" % ("-rotated" if nrot is not None else "", *cells, p)
    return Workload(name, tuple(cells), (1.0, 1.0, 2.0), p,
                    ("D", "N", "D", "D", "D", "D"), None, 1.0, f=gaussian((0.75, 0.5, 0.3)),
                    g=gaussian((0.0, 0.5, 0.5)), j=gaussian((1.0, 0.5, 0.5)), kfield=kfield, cfield=(0.0, 1e-8),
                    nrot=None if nrot is None else tuple(map(tuple, np.asarray(nrot, dtype=np.float64))))


def poisson_gauss(p=3, cells=None) -> Workload:
    """First diffusion test of Sec. 4.2: -lap u = f on [0,1] x [0,1] x [0,2],
    homogeneous Dirichlet, f a Gaussian of width 0.1 at (0.75, 0.5, 0.3);
    default grid: the paper's isotropic grid for degree p."""
    if cells is None:
        cells = {1: (128, 128, 256), 2: (56, 56, 112), 3: (32, 32, 64), 4: (20, 20, 40)}[p]
    return Workload("poisson-gauss-%dx%dx%d-p%d" % (*cells, p), tuple(cells), (1.0, 1.0, 2.0), p, ("D",) * 6, None,
                    1.0, f=gaussian((0.75, 0.5, 0.3)))


def w5_requests(n: int = 256, seed: int = 55):
    """The serving mix: list of (N, p, seed_i)."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([8, 12, 16, 24, 32], size=n)
    ps = rng.choice([2, 3, 4], size=n)
    return [(int(N), int(p), 5000 + i) for i, (N, p) in enumerate(zip(Ns, ps))]


def w5_problem(N: int, p: int, seed: int):
    rng = np.random.default_rng(seed)
    ncell = N**3
    K = np.exp(rng.normal(size=ncell))
    K = np.stack([K, K, K], axis=1)
    rhs = rng.normal(size=ncell * (p + 1) ** 3)
    return Workload(f"serve-{N}^3-p{p}", (N, N, N), (1.0, 1.0, 1.0), p, ("D",) * 6, None, K), rhs


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=n)


def random_case(p: int, cells=(5, 3, 4), seed: int = 0, with_b: bool = False, with_c: bool = True,
                bc=("D", "N", "D", "D", "N", "D"), lengths=(1.0, 0.7, 1.3), sigma=None) -> Workload:
    """Small random case with the structure of the workloads: random
    per-cell diagonal K (log-normal), optional reaction and affine advection,
    mixed boundary types."""
    rng = np.random.default_rng(seed)
    nc = int(np.prod(cells))
    K = np.exp(rng.normal(size=(nc, 3)))
    c = np.abs(rng.normal(size=nc)) if with_c else 0.0
    kw = {}
    if with_b:
        kw = dict(b0=(0.3, -0.7, 0.2), B=((0.5, 1.0, 0.0), (-1.0, -0.2, 0.5), (0.3, 0.0, -0.3)))
    return Workload(f"random-p{p}", cells, lengths, p, bc, sigma, K, c, **kw)
