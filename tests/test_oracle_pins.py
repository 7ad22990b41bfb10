"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an independent element-loop assembly with a dense inverse, a LAPACK
routine, the discrete maximum principle, exact scaling laws, symmetries of the
mesh, or brute-force point location.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from workload import rhs_nodal
from workload.gen import coefficient_field


def _rand_kappa(n, seed, var=1.0, corr=0.2, n_z=10):
    z = np.random.default_rng(seed).standard_normal((1, n_z))
    return coefficient_field(n, z, var, corr)[0]


def _rand_tri_kappa(n, seed, lo=0.1, hi=10.0):
    """Independent random value in every triangle (catches T-/T+ or index slips)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(n + 1, n + 1, 2))


# P1: exact discrete solution (closed form) -----------------------------------
@pytest.mark.parametrize("n", [7, 15, 63, 127])
def test_manufactured_exact_discrete(oracle_mod, n):
    O = oracle_mod
    k = np.ones((n + 1, n + 1, 2))
    u, rr = O.solve(n, k, rhs_nodal(n, "sinsin"))
    U = O.exact_discrete_sinsin(n)
    assert np.abs(u - U).max() / np.abs(U).max() < 1e-13
    assert rr < 1e-12


def test_manufactured_h2_convergence(oracle_mod):
    """Nodal error vs u = sin(pi x) sin(pi y) behaves like (pi h)^2/12 * u."""
    O = oracle_mod
    errs = []
    for n in [15, 31, 63]:
        h = 1.0 / (n + 1)
        u, _ = O.solve(n, np.ones((n + 1, n + 1, 2)), rhs_nodal(n, "sinsin"))
        x = np.arange(n + 2) * h
        X, Y = np.meshgrid(x, x)
        ue = np.sin(np.pi * X) * np.sin(np.pi * Y)
        e = np.abs(u - ue).max()
        errs.append(e)
        assert abs(e / ((np.pi * h) ** 2 / 12) - 1) < 0.05
    assert 3.9 < errs[0] / errs[1] < 4.1 and 3.9 < errs[1] / errs[2] < 4.1


# P2: dense brute force with independent element-loop assembly -------------------
@pytest.mark.parametrize("n,seed", [(1, 0), (3, 1), (5, 2), (7, 3), (7, 4)])
def test_dense_bruteforce(oracle_mod, n, seed):
    O = oracle_mod
    k = _rand_tri_kappa(n, seed)
    f = np.random.default_rng(100 + seed).uniform(-1, 2, size=(n + 2, n + 2))
    u, _ = O.solve(n, k, f)
    ud = O.dense_solve(n, k, f)
    assert np.abs(u - ud).max() / np.abs(ud).max() < 1e-13


@pytest.mark.parametrize("n", [3, 7, 15])
def test_band_equals_element_loop(oracle_mod, n):
    """The closed-form 5-point band equals the element-loop matrix (eq. coefA)."""
    O = oracle_mod
    k = _rand_tri_kappa(n, 7 + n)
    A, _, nodes = O.assemble_dense(n, k, np.zeros((n + 2, n + 2)))
    inner = [t for t, (i, j) in enumerate(nodes) if 1 <= i <= n and 1 <= j <= n]
    Ad = A[np.ix_(inner, inner)]
    B = O.band(n, k)
    full = np.zeros((n * n, n * n))
    for p in range(n * n):
        for d in range(n + 1):
            if p + d < n * n:
                full[p + d, p] = B[p, d]
                full[p, p + d] = B[p, d]
    assert np.abs(full - Ad).max() < 1e-13 * np.abs(Ad).max()


# P3: LAPACK banded Cholesky (scipy.linalg.solveh_banded) ------------------------
@pytest.mark.parametrize("n", [31, 63, 127])
def test_lapack_banded(oracle_mod, n):
    O = oracle_mod
    k = _rand_kappa(n, 11 + n, var=1.0, corr=0.1)
    f = rhs_nodal(n, "bump")
    u, _ = O.solve(n, k, f)
    B = O.band(n, k)  # lower form: B[p, d] = A[p+d, p]
    ab = np.ascontiguousarray(B.T)  # scipy lower form: ab[d, p] = A[p+d, p]
    x = scipy.linalg.solveh_banded(ab, O.load_vector(n, f), lower=True)
    assert np.abs(u[1:-1, 1:-1].reshape(-1) - x).max() / np.abs(x).max() < 1e-12


# P4: discrete maximum principle ---------------------------------------------------
def test_discrete_maximum_principle(oracle_mod):
    O = oracle_mod
    n = 31
    k = _rand_tri_kappa(n, 5, lo=1e-3, hi=1e3)
    f = np.random.default_rng(9).uniform(0.0, 1.0, size=(n + 2, n + 2))
    u, _ = O.solve(n, k, f)
    assert (u[1:-1, 1:-1] > 0).all()
    B = O.band(n, k)
    assert (B[:, 1:] <= 0).all()  # M-matrix off-diagonals


# P5: exact scaling laws ---------------------------------------------------------------
def test_kappa_scaling_bitwise(oracle_mod):
    """kappa -> 4 kappa scales the factor by exactly 2 and u by exactly 1/4."""
    O = oracle_mod
    n = 31
    k = _rand_kappa(n, 3)
    f = rhs_nodal(n, "bump")
    u1, _ = O.solve(n, k, f)
    u4, _ = O.solve(n, 4.0 * k, f)
    assert np.array_equal(u4 * 4.0, u1)


def test_kappa_constant(oracle_mod):
    O = oracle_mod
    n = 31
    u1, _ = O.solve(n, np.ones((n + 1, n + 1, 2)), rhs_nodal(n, "bump"))
    u3, _ = O.solve(n, 3.0 * np.ones((n + 1, n + 1, 2)), rhs_nodal(n, "bump"))
    assert np.abs(u3 * 3.0 - u1).max() < 1e-14 * np.abs(u1).max()


# P6: symmetries of the SW-NE mesh ---------------------------------------------------
def test_symmetry(oracle_mod):
    O = oracle_mod
    n = 63
    f = rhs_nodal(n, "one")
    u, _ = O.solve(n, np.ones((n + 1, n + 1, 2)), f)
    tol = 1e-13 * np.abs(u).max()
    assert np.abs(u - u.T).max() < tol          # (x, y) -> (y, x)
    assert np.abs(u - u[::-1, ::-1]).max() < tol  # 180 degree rotation


def test_transpose_symmetry_with_kappa(oracle_mod):
    """Reflection (x,y)->(y,x) maps T- of cell (i,j) to T+ of cell (j,i)."""
    O = oracle_mod
    n = 31
    k = _rand_tri_kappa(n, 21)
    kt = np.stack([k[:, :, 1].T, k[:, :, 0].T], axis=-1)
    f = np.random.default_rng(2).uniform(0, 1, size=(n + 2, n + 2))
    u, _ = O.solve(n, k, f)
    ut, _ = O.solve(n, kt, f.T.copy())
    assert np.abs(u.T - ut).max() < 1e-12 * np.abs(u).max()


# Refinement: accurate beyond cond * eps ------------------------------------------------
def test_refinement_high_contrast(oracle_mod):
    O = oracle_mod
    n = 15
    k = _rand_tri_kappa(n, 4, lo=1e-4, hi=1.0)
    f = rhs_nodal(n, "one")
    u0, _ = O.solve(n, k, f, sweeps=0)
    u2, rr = O.solve(n, k, f, sweeps=2)
    ud = O.dense_solve(n, k, f)
    assert np.abs(u2 - ud).max() / np.abs(ud).max() < 1e-12
    r = O.residual(n, k, f, u2)
    r0 = O.residual(n, k, f, u0)
    assert np.linalg.norm(r) <= np.linalg.norm(r0)
    assert rr < 1e-14


def test_residual_and_error_bound(oracle_mod):
    O = oracle_mod
    n = 31
    k = _rand_kappa(n, 8)
    f = rhs_nodal(n, "one")
    u, _ = O.solve(n, k, f)
    pert = np.zeros_like(u)
    pert[1:-1, 1:-1] = 1e-6 * np.random.default_rng(1).standard_normal((n, n))
    r = O.residual(n, k, f, u + pert)
    bound = O.error_bound_l2(n, k, r)
    assert np.linalg.norm(pert) <= bound * (1 + 1e-9)
    # smooth perturbation (lowest mode): the bound is tight up to the kappa ratio
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x)
    sm = 1e-6 * np.sin(np.pi * X) * np.sin(np.pi * Y)
    b2 = O.error_bound_l2(n, k, O.residual(n, k, f, u + sm))
    assert np.linalg.norm(sm) <= b2 * (1 + 1e-9) and b2 < 2 * np.linalg.norm(sm) * k.max() / k.min()


# P10: measurement operators ---------------------------------------------------------
def test_point_interpolation_affine(oracle_mod):
    O = oracle_mod
    n = 15
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x)
    u = 0.3 + 2.0 * X - 1.5 * Y
    pts = np.random.default_rng(0).uniform(size=(50, 2))
    pts = np.vstack([pts, [[0.0, 0.0], [1.0, 1.0], [0.5, 0.5], [1.0, 0.0], [3 * h, 3 * h], [1.0, 0.3]]])
    vals = O.point_values(n, u, pts)
    assert np.abs(vals - (0.3 + 2.0 * pts[:, 0] - 1.5 * pts[:, 1])).max() < 1e-13


def test_point_interpolation_bruteforce(oracle_mod):
    """Against a generic search over all triangles with barycentric coordinates."""
    O = oracle_mod
    n = 7
    h = 1.0 / (n + 1)
    u = np.random.default_rng(3).standard_normal((n + 2, n + 2))
    pts = np.random.default_rng(4).uniform(size=(40, 2))
    for p in pts:
        found = None
        for verts, _ in O._triangles(n, 0, n + 1, 0, n + 1):
            P = np.array([[v[0] * h, v[1] * h] for v in verts])
            M = np.array([[1, P[0, 0], P[0, 1]], [1, P[1, 0], P[1, 1]], [1, P[2, 0], P[2, 1]]]).T
            lam = np.linalg.solve(M, [1.0, p[0], p[1]])
            if (lam >= -1e-12).all():
                found = sum(lam[a] * u[verts[a][1], verts[a][0]] for a in range(3))
                break
        assert found is not None
        assert abs(found - O.point_value(n, u, p[0], p[1])) < 1e-12


def test_mean_and_interface(oracle_mod):
    O = oracle_mod
    n = 31
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x)
    u = 1.0 + 3.0 * X + 5.0 * Y
    m = O.mean_value(n, u, (0.25, 0.5, 0.25, 0.5))
    assert abs(m - (1.0 + 3.0 * 0.375 + 5.0 * 0.375)) < 1e-13
    # quadratic: exact integral of the P1 interpolant of x*y over [0,1/2]^2,
    # computed from the exact per-triangle rule with brute-force summation.
    u2 = X * Y
    ref = 0.0
    for verts, _ in O._triangles(n, 0, (n + 1) // 2, 0, (n + 1) // 2):
        vals = [u2[v[1], v[0]] for v in verts]
        ref += (h * h / 2) * sum(vals) / 3
    assert abs(O.mean_value(n, u2, (0.0, 0.5, 0.0, 0.5)) - ref / 0.25) < 1e-14
    iv = O.interface_values(n, u)
    assert np.allclose(iv, 1.0 + 1.5 + 5.0 * x[1:-1])


def test_node_interface(oracle_mod):
    """The interface of every tree node (eq. gamma_def) is the shared edge of
    its two sons without the edge's end points: every node on it lies on both
    sons' boundaries and strictly inside the father; |gamma| = cut length - 1;
    the root's is the midline.  Values are read off the affine field."""
    O = oracle_mod
    n, block = 63, 8
    nc = n + 1
    h = 1.0 / nc
    x = np.arange(nc + 1) * h
    X, Y = np.meshgrid(x, x)
    u = 1.0 + 3.0 * X + 5.0 * Y
    rects = O.tree_rects(n, block)
    n_inner = len(rects) - (nc // block) ** 2
    for k in range(n_inner):
        ids, vals = O.node_interface(n, u, block, k)
        i0, i1, j0, j1 = rects[k]
        sons = (rects[2 * k + 1], rects[2 * k + 2])
        assert len(ids) == (j1 - j0 - 1 if i1 - i0 >= j1 - j0 else i1 - i0 - 1)
        for q, v in zip(ids, vals):
            i, j = int(q % (nc + 1)), int(q // (nc + 1))
            assert i0 < i < i1 or j0 < j < j1
            assert i0 <= i <= i1 and j0 <= j <= j1
            for a0, a1, b0, b1 in sons:
                on_edge = (i in (a0, a1) and b0 <= j <= b1) or (j in (b0, b1) and a0 <= i <= a1)
                assert on_edge
            assert abs(v - (1.0 + 3.0 * i * h + 5.0 * j * h)) < 1e-13
    ids, vals = O.node_interface(n, u, block, 0)
    assert np.array_equal(vals, O.interface_values(n, u))


# P12: likelihood against scipy's normal log-density -------------------------------------
def test_loglik(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    hu = rng.standard_normal(20)
    y = hu + 0.01 * rng.standard_normal(20)
    sig = 0.01
    assert abs(O.loglik(y, hu, sig, normalized=True) - scipy.stats.norm.logpdf(y, hu, sig).sum()) < 1e-9
    assert O.loglik(hu, hu, sig) == 0.0
    assert abs(O.loglik(hu + 0.02, hu, sig) - (-20 * 0.02 ** 2 / (2 * sig ** 2))) < 1e-10


# Brute-force subdomain Schur complement (used to check per-node results) -----------------
def test_subdomain_schur_quotient(oracle_mod):
    """Schur complement of the whole domain onto the midline reproduces the
    global solution there (Section 2.4: u_1 solves the reduced system)."""
    O = oracle_mod
    n = 15
    nc = n + 1
    k = _rand_tri_kappa(n, 31)
    f = rhs_nodal(n, "bump")
    u, _ = O.solve(n, k, f)
    A, b, nodes = O.assemble_dense(n, k, f)
    mid = [t for t, (i, j) in enumerate(nodes) if i == nc // 2 and 1 <= j <= n]
    rest = [t for t, (i, j) in enumerate(nodes) if 1 <= i <= n and 1 <= j <= n and i != nc // 2]
    S = A[np.ix_(mid, mid)] - A[np.ix_(mid, rest)] @ np.linalg.solve(A[np.ix_(rest, rest)], A[np.ix_(rest, mid)])
    g = b[mid] - A[np.ix_(mid, rest)] @ np.linalg.solve(A[np.ix_(rest, rest)], b[rest])
    assert np.abs(np.linalg.solve(S, g) - O.interface_values(n, u)).max() < 1e-12 * np.abs(u).max()
    # floating subdomain: S 1 = 0, PSD; boundary-touching: PD
    Sf, _, _ = O.subdomain_schur(n, k, f, (4, 8, 4, 12))
    assert np.abs(Sf @ np.ones(len(Sf))).max() < 1e-12 * np.abs(Sf).max()
    ev = np.linalg.eigvalsh(Sf)
    assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]
    St, _, _ = O.subdomain_schur(n, k, f, (0, 8, 0, 8))
    assert np.linalg.eigvalsh(St)[0] > 0


# Subdomains of the tree and their means (Section 5.1) ----------------------------------
@pytest.mark.parametrize("n,block,count", [(63, 8, 127), (255, 16, 511), (1023, 16, 8191)])
def test_tree_rects_tile(oracle_mod, n, block, count):
    """Every depth tiles the square with 2^d equal halves of the depth above;
    the root is cut vertically at x = 1/2; the last depth is block x block."""
    O = oracle_mod
    nc = n + 1
    rects = O.tree_rects(n, block)
    assert len(rects) == count
    assert rects[0] == (0, nc, 0, nc) and rects[1] == (0, nc // 2, 0, nc) and rects[2] == (nc // 2, nc, 0, nc)
    start, d = 0, 0
    while start < len(rects):
        lev = rects[start:start + 2 ** d]
        cover = np.zeros((nc, nc), dtype=int)
        for i0, i1, j0, j1 in lev:
            cover[j0:j1, i0:i1] += 1
        assert (cover == 1).all()
        if d > 0:
            for k, (i0, i1, j0, j1) in enumerate(lev):
                fi0, fi1, fj0, fj1 = rects[start - 2 ** (d - 1) + k // 2]
                assert 2 * (i1 - i0) * (j1 - j0) == (fi1 - fi0) * (fj1 - fj0)
                assert fi0 <= i0 and i1 <= fi1 and fj0 <= j0 and j1 <= fj1
        start += 2 ** d
        d += 1
    assert all(r[1] - r[0] == block and r[3] - r[2] == block for r in rects[-(nc // block) ** 2:])


def test_node_means_root_closed_form(oracle_mod):
    """kappa = 1, f = 2 pi^2 sin sin: the P1 interpolant of the exact discrete
    solution U = C sin(pi x) sin(pi y) integrates to h^2 sum_p U_p (every
    interior node carries 6 triangles of area h^2/2, a third each), and
    sum_{i=1..N} sin(i pi h) = cot(pi h / 2), so the mean over the square is
    C h^2 cot^2(pi h / 2)."""
    O = oracle_mod
    for n in (15, 63):
        h = 1.0 / (n + 1)
        C = math.pi ** 2 * h * h / (4.0 * math.sin(math.pi * h / 2) ** 2)
        ref = C * h * h / math.tan(math.pi * h / 2) ** 2
        m = O.node_means(n, O.exact_discrete_sinsin(n), 8, nodes=[0])[0]
        assert abs(m - ref) < 1e-14 * abs(ref)


def test_node_means_sons_average(oracle_mod):
    """Means of the sons average to the father's mean with weights
    |omega_i| / |omega| (the constants c_1, c_2 of the example after Lemma
    Func1), at every node."""
    O = oracle_mod
    n = 63
    k = _rand_tri_kappa(n, 5)
    u, _ = O.solve(n, k, rhs_nodal(n, "bump"))
    rects = O.tree_rects(n, 8)
    m = O.node_means(n, u, 8)
    area = np.array([(r[1] - r[0]) * (r[3] - r[2]) for r in rects], dtype=float)
    for p in range((len(rects) - 1) // 2):
        a, b = 2 * p + 1, 2 * p + 2
        assert abs(m[p] - (area[a] * m[a] + area[b] * m[b]) / area[p]) < 1e-13 * np.abs(m).max()


@pytest.mark.parametrize("father", [(4, 12, 2, 10), (0, 16, 0, 16), (8, 16, 0, 8)])
def test_functional_lemma_dense(oracle_mod, father):
    """Lemma Func1 for the integral over a subdomain, brute force on dense
    matrices.  For a node with interior I and boundary Gamma, the integral of
    u_h is (l^f, f) + (l^g, u_Gamma) with l^g = w_Gamma - A_GI A_II^-1 w_I and
    (l^f, f) = w_I . A_II^-1 b_I, where w are the node's own quadrature weights
    (|t|/3 per triangle vertex, i.e. its load for f = 1).  The lemma builds
    both from the sons: with the son-union frame [gamma ; Gamma], the sum of
    the sons' Schur complements S~, loads g~ and functionals l~,
        l^g = l~_Gamma - S~_Gamma,gamma S~_gamma,gamma^-1 l~_gamma
        (l^f, f) = (l^f_1, f_1) + (l^f_2, f_2) + l~_gamma . S~_gamma,gamma^-1 g~_gamma
    (its last term uses l^g on gamma, as the lemma does).  Both must agree,
    and with u from the oracle give eq. mean times |omega|."""
    O = oracle_mod
    n = 15
    nc = n + 1
    h = 1.0 / nc
    k = _rand_tri_kappa(n, 77)
    f = rhs_nodal(n, "bump")
    ones = np.ones((n + 2, n + 2))
    u, _ = O.solve(n, k, f)
    i0, i1, j0, j1 = father
    if i1 - i0 >= j1 - j0:
        m = (i0 + i1) // 2
        sons = [(i0, m, j0, j1), (m, i1, j0, j1)]
    else:
        m = (j0 + j1) // 2
        sons = [(i0, i1, j0, m), (i0, i1, m, j1)]

    def direct(rect):
        S, g, bn = O.subdomain_schur(n, k, f, rect)
        _, lg, _ = O.subdomain_schur(n, k, ones, rect)
        A, b, nodes = O.assemble_dense(n, k, f, rect)
        _, w, _ = O.assemble_dense(n, k, ones, rect)
        a0, a1, b0, b1 = rect
        inner = [t for t, (i, j) in enumerate(nodes) if a0 < i < a1 and b0 < j < b1]
        mu = w[inner] @ np.linalg.solve(A[np.ix_(inner, inner)], b[inner]) if inner else 0.0
        return S, g, lg, mu, bn

    S_f, _, lg_f, mu_f, bn_f = direct(father)
    frame = {}
    parts = [direct(r) for r in sons]
    for _, _, _, _, bn in parts:
        for nd in bn:
            frame.setdefault(nd, len(frame))
    Uf = len(frame)
    St, gt, lt = np.zeros((Uf, Uf)), np.zeros(Uf), np.zeros(Uf)
    for S, g, lg, _, bn in parts:
        ix = [frame[nd] for nd in bn]
        St[np.ix_(ix, ix)] += S
        gt[ix] += g
        lt[ix] += lg
    G = [frame[nd] for nd in bn_f]
    gam = [t for nd, t in frame.items() if nd not in set(bn_f)]
    assert len(gam) > 0
    Sgg = St[np.ix_(gam, gam)]
    lam = lt[G] - St[np.ix_(G, gam)] @ np.linalg.solve(Sgg, lt[gam])
    mu = parts[0][3] + parts[1][3] + lt[gam] @ np.linalg.solve(Sgg, gt[gam])
    assert len(lam) == len(lg_f)
    if len(lg_f):
        assert np.abs(lam - lg_f).max() < 1e-12 * np.abs(lg_f).max()
    assert abs(mu - mu_f) < 1e-12 * abs(mu_f)
    ub = np.array([u[j, i] for i, j in bn_f]) if bn_f else np.zeros(0)
    integral = mu + lam @ ub
    area = (i1 - i0) * (j1 - j0) * h * h
    ref = O.mean_value(n, u, (i0 / nc, i1 / nc, j0 / nc, j1 / nc)) * area
    assert abs(integral - ref) < 1e-12 * abs(ref)


# Non-zero Dirichlet data ----------------------------------------------------------------
def test_dirichlet_affine_exact(oracle_mod):
    """Constant kappa, f = 0, affine boundary data: the P1 space holds the
    affine function, and it is discrete-harmonic (the gradients of a node's
    hat function sum to zero over its patch), so u_h equals it at every node."""
    O = oracle_mod
    n = 31
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x)
    g = 0.5 + 2.0 * X - 3.0 * Y
    u = O.solve_dirichlet(n, 2.5 * np.ones((n + 1, n + 1, 2)), np.zeros((n + 2, n + 2)), g)
    assert np.abs(u - g).max() < 1e-13


@pytest.mark.parametrize("n,seed", [(3, 1), (7, 2)])
def test_dirichlet_bruteforce(oracle_mod, n, seed):
    """Dense element-loop assembly on every node, boundary values moved to
    the right-hand side, inverse by LAPACK."""
    O = oracle_mod
    rng = np.random.default_rng(seed)
    k = _rand_tri_kappa(n, seed)
    f = rng.standard_normal((n + 2, n + 2))
    g = rng.standard_normal((n + 2, n + 2))
    A, b, nodes = O.assemble_dense(n, k, f)
    nc = n + 1
    inner = [t for t, (i, j) in enumerate(nodes) if 1 <= i <= n and 1 <= j <= n]
    bnd = [t for t, (i, j) in enumerate(nodes) if not (1 <= i <= n and 1 <= j <= n)]
    gD = np.array([g[nodes[t][1], nodes[t][0]] for t in bnd])
    uI = np.linalg.solve(A[np.ix_(inner, inner)], b[inner] - A[np.ix_(inner, bnd)] @ gD)
    u = O.solve_dirichlet(n, k, f, g)
    ref = g.copy()
    for t, val in zip(inner, uI):
        ref[nodes[t][1], nodes[t][0]] = val
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()
    assert nc == n + 1


def test_dirichlet_superposition(oracle_mod):
    """u(f, g) = u(f, 0) + u(0, g) (the operators F_h and G_h of eq.
    oper_represent2 are linear), and u(f, 0) is the zero-Dirichlet solve."""
    O = oracle_mod
    n = 31
    rng = np.random.default_rng(4)
    k = _rand_tri_kappa(n, 9)
    f = rhs_nodal(n, "bump")
    g = rng.uniform(-1, 1, (n + 2, n + 2))
    z = np.zeros((n + 2, n + 2))
    u = O.solve_dirichlet(n, k, f, g)
    u0, _ = O.solve(n, k, f)
    assert np.abs(O.solve_dirichlet(n, k, f, z) - u0).max() < 1e-14 * np.abs(u0).max()
    ug = O.solve_dirichlet(n, k, z, g)
    assert np.abs(u - (u0 + ug)).max() < 1e-13 * np.abs(u).max()


# Coarse-mesh data (Section 3.5) ----------------------------------------------------------
def test_prolong_affine_and_interpolant(oracle_mod):
    """The fine-mesh values of a coarse P1 function: affine functions are
    reproduced exactly, and the fine P1 interpolant of the prolonged values
    equals the coarse P1 function at arbitrary points (same SW-NE diagonals
    on both meshes)."""
    O = oracle_mod
    nH = 15
    m = nH + 1
    X, Y = np.meshgrid(np.arange(m + 1) / m, np.arange(m + 1) / m)
    fine = O.prolong(nH, 1.0 + 2.0 * X - 0.5 * Y)
    Xf, Yf = np.meshgrid(np.arange(2 * m + 1) / (2 * m), np.arange(2 * m + 1) / (2 * m))
    assert np.abs(fine - (1.0 + 2.0 * Xf - 0.5 * Yf)).max() < 1e-15
    rng = np.random.default_rng(3)
    v = rng.standard_normal((m + 1, m + 1))
    vf = O.prolong(nH, v)
    nh = 2 * m - 1
    for x, y in rng.uniform(0, 1, (200, 2)):
        assert abs(O.point_value(nh, vf, x, y) - O.point_value(nH, v, x, y)) < 1e-14
