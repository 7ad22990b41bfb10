"""Oracle for the HDD hot path: plain FP64 CPU reference.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the GPU library and
never imports it.

Contents
  solve(n, kappa, f)             global P1 solve, banded Cholesky + extended-
                                 precision refinement (oracle.c)
  solve_dirichlet(n, kappa, f, g)  the same with non-zero Dirichlet data
  lifted_load(n, kappa, f, g)    its interior load, as a nodal f
  prolong(n_coarse, v)           P1 values of a coarse-mesh function on the mesh of half the step
  residual(n, kappa, f, u)       b - A u in extended precision (oracle.c)
  point_values / interface / mean / loglik    the measurement operators
  tree_rects / node_means        subdomains of the tree and their means
  node_interface                 u on the interface gamma of one tree node
  element_matrix_dense(...)      independent element-loop assembly (dense)
  subdomain_schur(...)           brute-force dense Schur complement of one
                                 subdomain's own matrix (Section 2.4)

Every routine states the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O3, no fast-math, no machine-specific flags)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-o", _SO, src, "-lm"])
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_solve.restype = ctypes.c_int64
        lib.oracle_solve.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp]
        lib.oracle_residual.restype = None
        lib.oracle_residual.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        lib.oracle_band.restype = None
        lib.oracle_band.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_factor_prefix_seconds.restype = ctypes.c_double
        lib.oracle_factor_prefix_seconds.argtypes = [ctypes.c_int, dp, ctypes.c_int64]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Global solve (the FE solution the HDD result equals; abstract, Section 3.3)
# ---------------------------------------------------------------------------
def solve(n: int, kappa: np.ndarray, f: np.ndarray, sweeps: int = 2) -> Tuple[np.ndarray, float]:
    """u_full[j, i] (i, j in 0..N+1, zero on the boundary) and ||b-Au||/||b||."""
    lib = _load()
    k = _c(kappa).reshape(-1)
    assert k.size == 2 * (n + 1) ** 2
    ff = _c(f)
    assert ff.shape == (n + 2, n + 2)
    u = np.zeros((n + 2, n + 2))
    rr = ctypes.c_double(0.0)
    info = lib.oracle_solve(n, _p(k), _p(ff), int(sweeps), _p(u), ctypes.byref(rr))
    if info != 0:
        raise RuntimeError(f"oracle_solve failed: info={info}")
    return u, rr.value


def lifted_load(n: int, kappa: np.ndarray, f: np.ndarray, g: np.ndarray) -> np.ndarray:
    """The nodal load f' whose interior load vector is b_I - A_ID g_D (u = g
    on the outer boundary, eq. elliptic_det): the lifting A_ID g_D is summed
    triangle by triangle from the element matrices of eq. coefA over the ring
    of cells that touches the boundary, and divided by h^2 (the load vector
    of eq. coefc is h^2 f at an interior node)."""
    nc = n + 1
    h = 1.0 / nc
    k = np.asarray(kappa, dtype=np.float64).reshape(nc, nc, 2)
    gg = np.asarray(g, dtype=np.float64)

    def boundary(v):
        return v[0] in (0, nc) or v[1] in (0, nc)

    lift = np.zeros((n + 2, n + 2))
    ring = [(i, j) for j in range(nc) for i in range(nc) if i in (0, nc - 1) or j in (0, nc - 1)]
    for i, j in ring:
        for verts, (jj, ii, t) in _triangles(n, i, i + 1, j, j + 1):
            K, _ = _element(verts, k[jj, ii, t], h)
            for a in range(3):
                if boundary(verts[a]):
                    continue
                for c in range(3):
                    if boundary(verts[c]):
                        lift[verts[a][1], verts[a][0]] += K[a, c] * gg[verts[c][1], verts[c][0]]
    return np.asarray(f, dtype=np.float64) - lift / (h * h)


def prolong(n_coarse: int, v: np.ndarray) -> np.ndarray:
    """Nodal values on the mesh of step h = H/2 of the P1 function with nodal
    values v on the coarse mesh of step H (Section 3.5, multiple scales: a
    smooth right-hand side given on a coarser mesh).  Both meshes split every
    cell along its SW-NE diagonal, so a fine node is a coarse node, the
    midpoint of a horizontal or vertical coarse edge, or the midpoint of a
    coarse diagonal, and takes the coarse value or the mean of the edge's two
    ends.  v: [n_coarse+2]^2; returns [2 n_coarse + 3]^2."""
    v = np.asarray(v, dtype=np.float64)
    m = n_coarse + 1  # coarse cells per side
    out = np.zeros((2 * m + 1, 2 * m + 1))
    for J in range(m + 1):
        for I in range(m + 1):
            out[2 * J, 2 * I] = v[J, I]
            if I < m:
                out[2 * J, 2 * I + 1] = 0.5 * (v[J, I] + v[J, I + 1])
            if J < m:
                out[2 * J + 1, 2 * I] = 0.5 * (v[J, I] + v[J + 1, I])
            if I < m and J < m:
                out[2 * J + 1, 2 * I + 1] = 0.5 * (v[J, I] + v[J + 1, I + 1])
    return out


def solve_dirichlet(n: int, kappa: np.ndarray, f: np.ndarray, g: np.ndarray, sweeps: int = 2) -> np.ndarray:
    """u_full for the problem with Dirichlet data: u = g at the outer boundary
    nodes and, inside, the zero-Dirichlet solve above with the lifted load."""
    gg = np.asarray(g, dtype=np.float64)
    u, _ = solve(n, kappa, lifted_load(n, kappa, f, g), sweeps)
    u[0, :], u[-1, :], u[:, 0], u[:, -1] = gg[0, :], gg[-1, :], gg[:, 0], gg[:, -1]
    return u


def residual(n: int, kappa: np.ndarray, f: np.ndarray, u_full: np.ndarray) -> np.ndarray:
    """(b - A u) on the nodal grid, extended-precision accumulation."""
    lib = _load()
    k = _c(kappa).reshape(-1)
    ff = _c(f)
    uu = _c(u_full)
    r = np.zeros((n + 2, n + 2))
    lib.oracle_residual(n, _p(k), _p(ff), _p(uu), _p(r))
    return r


def band(n: int, kappa: np.ndarray) -> np.ndarray:
    """Lower band of A, column-major: out[p, d] = A[p+d, p]."""
    lib = _load()
    k = _c(kappa).reshape(-1)
    out = np.zeros((n * n, n + 1))
    lib.oracle_band(n, _p(k), _p(out))
    return out


def factor_prefix_seconds(n: int, kappa: np.ndarray, ncols: int) -> float:
    lib = _load()
    k = _c(kappa).reshape(-1)
    t = lib.oracle_factor_prefix_seconds(n, _p(k), int(ncols))
    if t < 0:
        raise RuntimeError("oracle factor prefix failed")
    return t


def load_vector(n: int, f: np.ndarray) -> np.ndarray:
    """b_p = sum over the 6 triangles at p of |t| f_p / 3 (eq. coefc)."""
    h = 1.0 / (n + 1)
    return (6.0 * (0.5 * h * h) * np.asarray(f, dtype=np.float64) / 3.0)[1:-1, 1:-1].reshape(-1)


# ---------------------------------------------------------------------------
# Measurement operators (Section 1.2 examples; Section 5 eq. mean)
# ---------------------------------------------------------------------------
def point_value(n: int, u_full: np.ndarray, x: float, y: float) -> float:
    """P1 interpolation of the nodal field at (x, y) in the unit square.

    The cell is ci = min(floor(x/h), N), fx = x/h - ci (same for y).  If
    fx >= fy the point is in T- with barycentric weights (1-fx, fx-fy, fy) at
    (ci,cj), (ci+1,cj), (ci+1,cj+1); else in T+ with weights (1-fy, fx, fy-fx)
    at (ci,cj), (ci+1,cj+1), (ci,cj+1).
    """
    nc = n + 1
    ci = min(int(math.floor(x * nc)), n)
    cj = min(int(math.floor(y * nc)), n)
    fx = x * nc - ci
    fy = y * nc - cj
    u = u_full
    if fx >= fy:
        return (1 - fx) * u[cj, ci] + (fx - fy) * u[cj, ci + 1] + fy * u[cj + 1, ci + 1]
    return (1 - fy) * u[cj, ci] + fx * u[cj + 1, ci + 1] + (fy - fx) * u[cj + 1, ci]


def point_values(n: int, u_full: np.ndarray, pts: np.ndarray) -> np.ndarray:
    return np.array([point_value(n, u_full, float(p[0]), float(p[1])) for p in np.atleast_2d(pts)])


def interface_values(n: int, u_full: np.ndarray) -> np.ndarray:
    """u on the root interface, the vertical midline x = 1/2: nodes (Nc/2, j), j = 1..N."""
    nc = n + 1
    assert nc % 2 == 0
    return np.array(u_full[1:n + 1, nc // 2])


def mean_value(n: int, u_full: np.ndarray, rect: Sequence[float]) -> float:
    """eq. mean: sum over triangles t in R of (|t|/3)(u1+u2+u3), divided by |R|.

    rect = (x0, x1, y0, y1) aligned with cell boundaries.
    """
    nc = n + 1
    h = 1.0 / nc
    i0, i1 = int(round(rect[0] * nc)), int(round(rect[1] * nc))
    j0, j1 = int(round(rect[2] * nc)), int(round(rect[3] * nc))
    area_t = 0.5 * h * h
    total = 0.0
    for j in range(j0, j1):
        for i in range(i0, i1):
            a, b, c, d = u_full[j, i], u_full[j, i + 1], u_full[j + 1, i + 1], u_full[j + 1, i]
            total += area_t / 3.0 * (a + b + c)  # T-
            total += area_t / 3.0 * (a + c + d)  # T+
    return total / ((i1 - i0) * (j1 - j0) * h * h)


def tree_rects(n: int, block: int) -> list:
    """Cell rectangles (i0, i1, j0, j1) of every node of the HDD tree (Section
    2.1) down to block x block cells, root first, then depth by depth, each
    father's two sons next to each other (left before right for a vertical
    cut, bottom before top for a horizontal one).  The paper only asks for
    halves with a small shared interface; the split taken here cuts the longer
    side at its midpoint and cuts squares vertically, so the root interface is
    the midline x = 1/2."""
    nc = n + 1
    level = [(0, nc, 0, nc)]
    out = list(level)
    while level[0][1] - level[0][0] > block or level[0][3] - level[0][2] > block:
        nxt = []
        for i0, i1, j0, j1 in level:
            if i1 - i0 >= j1 - j0:
                m = (i0 + i1) // 2
                nxt += [(i0, m, j0, j1), (m, i1, j0, j1)]
            else:
                m = (j0 + j1) // 2
                nxt += [(i0, i1, j0, m), (i0, i1, m, j1)]
        level = nxt
        out += level
    return out


def node_interface(n: int, u_full: np.ndarray, block: int, k: int):
    """(ids, values) of u on the interface gamma of tree node k (order of
    tree_rects): the cut that splits the node's rectangle into its two sons
    without the cut's two end points (eq. gamma_def, Section 2.1), nodes in
    increasing coordinate along the cut; ids are j (Nc + 1) + i."""
    nc = n + 1
    i0, i1, j0, j1 = tree_rects(n, block)[k]
    if i1 - i0 >= j1 - j0:
        m = (i0 + i1) // 2
        nodes = [(m, j) for j in range(j0 + 1, j1)]
    else:
        m = (j0 + j1) // 2
        nodes = [(i, m) for i in range(i0 + 1, i1)]
    ids = np.array([j * (nc + 1) + i for i, j in nodes], dtype=np.int64)
    return ids, np.array([u_full[j, i] for i, j in nodes])


def node_means(n: int, u_full: np.ndarray, block: int, nodes=None) -> np.ndarray:
    """Mean of u_h over every subdomain of the tree (the example after Lemma
    Func1 in Section 5.1: mean values in all subdomains), each by eq. mean
    over the node's own triangles, in the order of tree_rects.  nodes: indices
    into that order to evaluate (default all)."""
    nc = n + 1
    rects = tree_rects(n, block)
    pick = range(len(rects)) if nodes is None else nodes
    return np.array([mean_value(n, u_full, tuple(c / nc for c in rects[k])) for k in pick])


def loglik(y: np.ndarray, hu: np.ndarray, sigma: float, normalized: bool = False) -> float:
    """log of L(z) = prod_i pi_eps(y_i - S_i(z)) for Gaussian noise N(0, sigma^2)
    (likelihood formula at the end of Section 1.2)."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(hu, dtype=np.float64)
    val = -float(np.sum(r * r)) / (2.0 * sigma * sigma)
    if normalized:
        val -= r.size * math.log(sigma * math.sqrt(2.0 * math.pi))
    return val


# ---------------------------------------------------------------------------
# Independent element-loop assembly and brute-force Schur complements
# ---------------------------------------------------------------------------
def _triangles(n: int, i0: int, i1: int, j0: int, j1: int):
    """Triangles (vertex node tuples, kappa index) of cells in [i0,i1) x [j0,j1)."""
    for j in range(j0, j1):
        for i in range(i0, i1):
            yield ((i, j), (i + 1, j), (i + 1, j + 1)), (j, i, 0)
            yield ((i, j), (i + 1, j + 1), (i, j + 1)), (j, i, 1)


def _element(verts, kap: float, h: float):
    """P1 element matrix of eq. coefA from vertex gradients: kappa |t| grad b_i . grad b_j."""
    P = np.array([[v[0] * h, v[1] * h] for v in verts])
    M = np.array([[1.0, P[0, 0], P[0, 1]], [1.0, P[1, 0], P[1, 1]], [1.0, P[2, 0], P[2, 1]]])
    area = 0.5 * abs(np.linalg.det(M))
    G = np.linalg.inv(M)[1:, :]  # gradients of the 3 barycentric functions (columns)
    return kap * area * (G.T @ G), area


def assemble_dense(n: int, kappa: np.ndarray, f: np.ndarray, rect_cells=None):
    """Element-loop assembly over the cells of rect_cells = (i0, i1, j0, j1)
    (default: all).  Returns (A, b, nodes) on every mesh node of the rectangle,
    nodes[k] = (i, j); b uses the vertex rule of eq. coefc per triangle."""
    nc = n + 1
    h = 1.0 / nc
    k = np.asarray(kappa).reshape(nc, nc, 2)
    i0, i1, j0, j1 = rect_cells if rect_cells is not None else (0, nc, 0, nc)
    nodes = [(i, j) for j in range(j0, j1 + 1) for i in range(i0, i1 + 1)]
    idx = {nd: t for t, nd in enumerate(nodes)}
    A = np.zeros((len(nodes), len(nodes)))
    b = np.zeros(len(nodes))
    for verts, (jj, ii, s) in _triangles(n, i0, i1, j0, j1):
        K, area = _element(verts, k[jj, ii, s], h)
        for a in range(3):
            pa = idx[verts[a]]
            b[pa] += area * f[verts[a][1], verts[a][0]] / 3.0
            for c in range(3):
                A[pa, idx[verts[c]]] += K[a, c]
    return A, b, nodes


def dense_solve(n: int, kappa: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Brute force for tiny grids: u = inv(A) b with element-loop assembly."""
    A, b, nodes = assemble_dense(n, kappa, f)
    inner = [t for t, (i, j) in enumerate(nodes) if 1 <= i <= n and 1 <= j <= n]
    u = np.linalg.inv(A[np.ix_(inner, inner)]) @ b[inner]
    out = np.zeros((n + 2, n + 2))
    for t, val in zip(inner, u):
        i, j = nodes[t]
        out[j, i] = val
    return out


def subdomain_schur(n: int, kappa: np.ndarray, f: np.ndarray, rect_cells, drop_dirichlet: bool = True):
    """Schur complement of a subdomain's own matrix onto its boundary (eq.
    SchurMinus1 / SchurC1 with block 1 = boundary, block 2 = interior):
        S = A_bb - A_bi A_ii^-1 A_ib,   g = b_b - A_bi A_ii^-1 b_i.
    The subdomain matrix is assembled from the triangles of the rectangle
    only.  Boundary nodes on the outer Dirichlet boundary are dropped when
    drop_dirichlet (their values are zero).  Returns (S, g, boundary_nodes)."""
    i0, i1, j0, j1 = rect_cells
    A, b, nodes = assemble_dense(n, kappa, f, rect_cells)
    nc = n + 1

    def on_rect_boundary(nd):
        return nd[0] in (i0, i1) or nd[1] in (j0, j1)

    def dirichlet(nd):
        return nd[0] in (0, nc) or nd[1] in (0, nc)

    inner = [t for t, nd in enumerate(nodes) if not on_rect_boundary(nd)]
    bnd = [t for t, nd in enumerate(nodes) if on_rect_boundary(nd) and not (drop_dirichlet and dirichlet(nd))]
    Aii = A[np.ix_(inner, inner)]
    Aib = A[np.ix_(inner, bnd)]
    Abi = A[np.ix_(bnd, inner)]
    S = A[np.ix_(bnd, bnd)] - Abi @ np.linalg.solve(Aii, Aib) if inner else A[np.ix_(bnd, bnd)]
    g = b[bnd] - Abi @ np.linalg.solve(Aii, b[inner]) if inner else b[bnd]
    return S, g, [nodes[t] for t in bnd]


def exact_discrete_sinsin(n: int) -> np.ndarray:
    """Closed-form discrete solution for kappa = 1, f = 2 pi^2 sin(pi x) sin(pi y).

    sin(pi x) sin(pi y) is an eigenvector of the unit 5-point operator with
    eigenvalue 8 sin^2(pi h / 2); with b = h^2 f the nodal solution is
    U = pi^2 h^2 / (4 sin^2(pi h/2)) sin(pi x) sin(pi y)."""
    nc = n + 1
    h = 1.0 / nc
    x = np.arange(nc + 1) * h
    X, Y = np.meshgrid(x, x)
    U = (math.pi ** 2 * h * h) / (4.0 * math.sin(math.pi * h / 2) ** 2) * np.sin(math.pi * X) * np.sin(math.pi * Y)
    U[0, :] = U[-1, :] = 0.0
    U[:, 0] = U[:, -1] = 0.0
    return U


def error_bound_l2(n: int, kappa: np.ndarray, r_full: np.ndarray) -> float:
    """Rigorous bound ||u - u_h||_2 <= ||r||_2 / lambda_min(A) with
    lambda_min(A) >= min(kappa) * 8 sin^2(pi h / 2): A is a sum of nonnegative
    multiples kappa_t of PSD element matrices, so A >= min(kappa) A_1, and
    A_1 (unit coefficient) is the 5-point Laplacian."""
    h = 1.0 / (n + 1)
    lam = float(np.min(kappa)) * 8.0 * math.sin(math.pi * h / 2) ** 2
    return float(np.linalg.norm(r_full)) / lam
