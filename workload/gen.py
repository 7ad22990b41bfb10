"""Seeded synthetic workloads for -div(kappa grad u) = f on the unit square.

Mesh convention (shared input format, not solver arithmetic): N interior nodes
per side, Nc = N + 1 cells per side, h = 1/Nc.  Cell (i, j) spans
[i h, (i+1) h] x [j h, (j+1) h] and is split along its SW-NE diagonal into
T- = {(i,j), (i+1,j), (i+1,j+1)} and T+ = {(i,j), (i+1,j+1), (i,j+1)}.
The coefficient is piecewise constant per triangle and stored as
kappa[s, j, i, 0] for T- and kappa[s, j, i, 1] for T+ (float64, C order).
The right-hand side is nodal, f[j, i] for i, j in 0..Nc (boundary entries are
carried but never used: the Dirichlet data is zero).

The coefficient model follows the paper's kappa(x, Z) = exp(q(x, Z)) with
independent standard-normal parameters Z (Section 1, notation table and
Bayesian updating subsection).  The paper does not fix the expansion of q; we
use a truncated Karhunen-Loeve-type sine expansion of a Gaussian covariance
c(r) = var * exp(-r^2 / (2 corr^2)):
    q(x) = sum_m sqrt(lam_m) * 2 sin(j_m pi x1) sin(k_m pi x2) * Z_m,
    lam_jk = var * 2 pi corr^2 * exp(-(j^2 + k^2) pi^2 corr^2 / 2),
keeping the n_z largest lam ordered by (j^2 + k^2, j).  kappa is evaluated at
triangle centroids ((i+2/3)h, (j+1/3)h) for T- and ((i+1/3)h, (j+2/3)h) for T+.

Seeding: rng = numpy.random.default_rng(seed); Z = rng.standard_normal((n_s,
n_z)); then observation sites = rng.uniform(size=(n_q, 2)).  The "true"
parameter behind synthetic observations is drawn from default_rng(seed + 1000):
Z_true = standard_normal(n_z), then noise = sigma_y * standard_normal(n_q).
Observations y = u_true(sites) + noise are formed by whoever holds a solver.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

# Workloads.  Sizes, coefficient statistics and query sets follow the
# benchmark configurations; seeds are the configuration index.
CONFIGS = {
    # plain single solve, 63^2 interior nodes, 8x8-cell leaves
    "c0_63": dict(n=63, leaf=8, var=0.5, corr=0.2, n_z=10, f="one", n_s=1,
                  n_q=5, sigma_y=0.01, seed=0, interface=False, mean_rect=None),
    # batched: 255^2 interior nodes, 16x16 leaves, 256 parameter samples
    "c1_255": dict(n=255, leaf=16, var=1.0, corr=0.1, n_z=20, f="one", n_s=256,
                   n_q=16, sigma_y=0.01, seed=1, interface=False, mean_rect=None),
    # large partial solve: 1023^2, 32x32 leaves; points + midline + a mean
    "c2_1023": dict(n=1023, leaf=32, var=1.0, corr=0.05, n_z=50, f="one", n_s=4,
                    n_q=64, sigma_y=0.01, seed=2, interface=True,
                    mean_rect=(0.25, 0.5, 0.25, 0.5)),
    # serving mix members (mesh drawn per request from these)
    "s_127": dict(n=127, leaf=16, var=1.0, corr=0.1, n_z=20, f="one", n_s=1,
                  n_q=32, sigma_y=0.01, seed=3, interface=False, mean_rect=None),
    "s_255": dict(n=255, leaf=16, var=1.0, corr=0.1, n_z=20, f="one", n_s=1,
                  n_q=32, sigma_y=0.01, seed=3, interface=False, mean_rect=None),
    "s_511": dict(n=511, leaf=16, var=1.0, corr=0.1, n_z=20, f="one", n_s=1,
                  n_q=32, sigma_y=0.01, seed=3, interface=False, mean_rect=None),
    # high-contrast stress: 2047^2, variance 4, corr 0.02, 200 modes, bump rhs
    "c4_2047": dict(n=2047, leaf=32, var=4.0, corr=0.02, n_z=200, f="bump",
                    n_s=1, n_q=128, sigma_y=0.01, seed=4, interface=True,
                    mean_rect=None),
}


def kl_modes(n_z: int, var: float, corr: float):
    """(j, k, lam) of the n_z largest sine modes, ordered by (j^2+k^2, j)."""
    cand = [(j * j + k * k, j, k) for j in range(1, n_z + 2) for k in range(1, n_z + 2)]
    cand.sort()
    sel = cand[:n_z]
    j = np.array([c[1] for c in sel], dtype=np.float64)
    k = np.array([c[2] for c in sel], dtype=np.float64)
    lam = var * 2.0 * np.pi * corr ** 2 * np.exp(-(j * j + k * k) * np.pi ** 2 * corr ** 2 / 2.0)
    return j, k, lam


def _centroids(n: int):
    nc = n + 1
    h = 1.0 / nc
    i = np.arange(nc, dtype=np.float64)
    # T-: ((i+2/3)h, (j+1/3)h); T+: ((i+1/3)h, (j+2/3)h)
    return h, (i + 2.0 / 3.0) * h, (i + 1.0 / 3.0) * h


def coefficient_field(n: int, z: np.ndarray, var: float, corr: float) -> np.ndarray:
    """log-normal kappa per triangle, shape [n_s, Nc, Nc, 2], float64."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    n_s, n_z = z.shape
    jm, km, lam = kl_modes(n_z, var, corr)
    _, a23, a13 = _centroids(n)
    coef = 2.0 * np.sqrt(lam)[None, :] * z  # [n_s, n_z]
    # T-: x at (i+2/3)h, y at (j+1/3)h
    sx_m = np.sin(np.pi * jm[:, None] * a23[None, :])  # [n_z, Nc]
    sy_m = np.sin(np.pi * km[:, None] * a13[None, :])
    # T+: x at (i+1/3)h, y at (j+2/3)h
    sx_p = np.sin(np.pi * jm[:, None] * a13[None, :])
    sy_p = np.sin(np.pi * km[:, None] * a23[None, :])
    nc = n + 1
    out = np.empty((n_s, nc, nc, 2), dtype=np.float64)
    for s in range(n_s):
        q_m = (sy_m.T * coef[s][None, :]) @ sx_m  # [j, i]
        q_p = (sy_p.T * coef[s][None, :]) @ sx_p
        out[s, :, :, 0] = np.exp(q_m)
        out[s, :, :, 1] = np.exp(q_p)
    return out


def edge_sites(n: int) -> np.ndarray:
    """Observation sites on the places where locating the holding triangle is
    delicate, shape [m, 2]: the corners and edges of the unit square, the
    root midline x = 1/2 and the line y = 1/2, lines x or y = k * 16 h
    (boundaries of 16 x 16-cell blocks and of the leaves above them), exact
    mesh nodes (block corners among them), and points on cell diagonals
    (fx = fy).  Cells have the dyadic side h = 1/(N+1), so every coordinate
    here is exact in binary."""
    nc = n + 1
    h = 1.0 / nc
    q = nc // 4
    pts = [(0.0, 0.0), (1.0, 1.0), (0.0, 1.0), (1.0, 0.0), (0.0, 0.375), (1.0, 0.625), (0.3125, 0.0),
           (0.6875, 1.0), (0.5, 0.5), (0.5, 0.125), (0.5, 1.0 - h), (0.75, 0.5), (h, 0.5)]
    # exact mesh nodes, block and leaf corners among them
    for i, j in ((1, 1), (nc - 1, nc - 1), (min(16, nc - 1), min(16, nc - 1)), (nc // 2, q), (q, 3 * q),
                 (min(17, nc - 1), min(33, nc - 1)), (nc // 2 - 1, nc // 2 + 1)):
        pts.append((i * h, j * h))
    # block / leaf boundaries off the nodes: x or y a multiple of 16 h
    for k in sorted({min(16, nc // 2), nc // 2, q, 3 * q}):
        pts.append((k * h, (k // 2 + 0.375) * h))
        pts.append(((k // 2 + 0.625) * h, k * h))
    # cell diagonals, fx == fy
    for i, j, t in ((5, 9, 0.25), (nc // 2 - 1, q, 0.5), (q, nc // 2, 0.75), (nc - 2, 3, 0.5)):
        pts.append(((i + t) * h, (j + t) * h))
    return np.array(pts, dtype=np.float64)


def off_tree_rects(n: int):
    """Cell-aligned rectangles (x0, x1, y0, y1) that are not nodes of the
    tree: one crossing the root midline and the line y = 1/2, one thin strip
    on the outer boundary, and a small one (inside one 16 x 16-cell block
    when N + 1 >= 128)."""
    nc = n + 1
    h = 1.0 / nc
    q = nc // 4
    return [((3) * h, (nc // 2 + 5) * h, (nc // 8 + 1) * h, (3 * q - 3) * h),
            (0.0, 1.0, 0.0, 2 * h),
            ((q + 2) * h, (q + 9) * h, (q + 4) * h, (q + 6) * h)]


def kappa_from_q(q_minus: np.ndarray, q_plus: np.ndarray) -> np.ndarray:
    """Stack per-triangle log-coefficients [Nc, Nc] into kappa [1, Nc, Nc, 2]."""
    return np.exp(np.stack([q_minus, q_plus], axis=-1))[None]


def paper_kappa(n: int, kind: str) -> np.ndarray:
    """Deterministic coefficients used in the paper's numerical section.

    "sin50":  kappa = 1 + 0.5 sin(50x) sin(50y)
    "alpha500": alpha = 1 / (1.0001 + sin(500x) sin(500y))
    evaluated at triangle centroids; shape [1, Nc, Nc, 2].
    """
    _, a23, a13 = _centroids(n)
    xm, ym = np.meshgrid(a23, a13)  # T-: [j, i]
    xp, yp = np.meshgrid(a13, a23)  # T+
    if kind == "sin50":
        fm = 1.0 + 0.5 * np.sin(50 * xm) * np.sin(50 * ym)
        fp = 1.0 + 0.5 * np.sin(50 * xp) * np.sin(50 * yp)
    elif kind == "alpha500":
        fm = 1.0 / (1.0001 + np.sin(500 * xm) * np.sin(500 * ym))
        fp = 1.0 / (1.0001 + np.sin(500 * xp) * np.sin(500 * yp))
    else:
        raise ValueError(kind)
    return np.stack([fm, fp], axis=-1)[None].copy()


def rhs_nodal(n: int, kind: str = "one") -> np.ndarray:
    """Nodal right-hand side f[j, i], i, j in 0..Nc, float64."""
    nc = n + 1
    x = np.arange(nc + 1, dtype=np.float64) / nc
    X, Y = np.meshgrid(x, x)  # [j, i]
    if kind == "one":
        return np.ones((nc + 1, nc + 1), dtype=np.float64)
    if kind == "bump":
        return np.exp(-((X - 0.3) ** 2 + (Y - 0.7) ** 2) / (2 * 0.05 ** 2))
    if kind == "sinsin":
        return 2.0 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(np.pi * Y)
    raise ValueError(kind)


@dataclass
class Workload:
    name: str
    n: int
    leaf: int
    kappa: np.ndarray            # [n_s, Nc, Nc, 2]
    f: np.ndarray                # [Nc+1, Nc+1]
    z: np.ndarray                # [n_s, n_z]
    points: np.ndarray           # [n_q, 2]
    sigma_y: float
    z_true: np.ndarray           # [n_z]
    kappa_true: np.ndarray       # [1, Nc, Nc, 2]
    noise: np.ndarray            # [n_q]
    interface: bool = False
    mean_rect: Optional[Tuple[float, float, float, float]] = None
    spec: dict = field(default_factory=dict)


def make_workload(name: str, n_samples: Optional[int] = None, with_true: bool = True) -> Workload:
    spec = dict(CONFIGS[name])
    if n_samples is not None:
        spec["n_s"] = int(n_samples)
    n, n_z = spec["n"], spec["n_z"]
    # The configuration's own sample count fixes the stream position of the
    # observation sites; extra samples are drawn after the sites.
    n_base = CONFIGS[name]["n_s"]
    rng = np.random.default_rng(spec["seed"])
    z = rng.standard_normal((n_base, n_z))
    points = rng.uniform(size=(spec["n_q"], 2))
    if spec["n_s"] > n_base:
        z = np.concatenate([z, rng.standard_normal((spec["n_s"] - n_base, n_z))])
    z = z[: spec["n_s"]]
    trng = np.random.default_rng(spec["seed"] + 1000)
    z_true = trng.standard_normal(n_z)
    noise = spec["sigma_y"] * trng.standard_normal(spec["n_q"])
    kappa = coefficient_field(n, z, spec["var"], spec["corr"])
    kappa_true = coefficient_field(n, z_true[None], spec["var"], spec["corr"]) if with_true else None
    return Workload(name=name, n=n, leaf=spec["leaf"], kappa=kappa, f=rhs_nodal(n, spec["f"]),
                    z=z, points=points, sigma_y=spec["sigma_y"], z_true=z_true,
                    kappa_true=kappa_true, noise=noise, interface=spec["interface"],
                    mean_rect=spec["mean_rect"], spec=spec)
