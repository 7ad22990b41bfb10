"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (normwise, ||v - v_oracle||_inf / ||v_oracle||_inf):
  HDD_FP64          1e-10
  HDD_FP32_REFINE   1e-8
"""
import sys

import numpy as np
import pytest

try:  # import at collection so a slow first import is not charged to a test
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

from workload import make_workload, rhs_nodal
from workload.gen import coefficient_field

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_02207_amd import hdd
    return hdd


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_values(O, n, kappa, f, pts, rect=None):
    u, _ = O.solve(n, kappa, f)
    out = dict(u=u, pts=O.point_values(n, u, pts), iface=O.interface_values(n, u))
    if rect is not None:
        out["mean"] = O.mean_value(n, u, rect)
    return out


def test_mfma_lane_layout(H):
    say("mfma selftest")
    for dtype, n, kdim in [(0, 32, 8), (1, 16, 8)]:
        out = H.hdd_mfma_selftest(dtype)
        i = np.arange(n)[:, None]
        k = np.arange(kdim)[None, :]
        A = ((i * 7 + k * 3) % 11) - 5.0
        B = ((i * 5 + k * 2) % 13) - 6.0
        assert np.array_equal(out, A @ B.T), dtype


@pytest.mark.parametrize("flags", [0, 1])
def test_c0_fp64(H, oracle_mod, flags):
    """63^2, 8x8 leaves, one sample: points, midline interface, mean."""
    w = make_workload("c0_63")
    say("c0_63 fp64 flags", flags)
    o = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf, flags=flags)
    t = H.HDD(o, 1)
    t.build(w.kappa, w.f)
    rect = (0.25, 0.5, 0.25, 0.5)
    ref = oracle_values(oracle_mod, w.n, w.kappa[0], w.f, w.points, rect)
    got = t.query_points(w.points)[0]
    assert rel(got, ref["pts"]) < TOL64
    assert rel(t.query_interface()[0], ref["iface"]) < TOL64
    assert rel(t.query_mean(rect), [ref["mean"]]) < TOL64
    t.solve_full()
    assert rel(t.solution(0), ref["u"]) < TOL64
    t.close()


@pytest.mark.parametrize("n,leaf,flags", [(3, 2, 1), (15, 4, 1), (15, 4, 0), (31, 4, 1), (63, 8, 1)])
def test_node_schur_bruteforce(H, oracle_mod, n, leaf, flags):
    """Per-node S_omega and g_omega equal the dense Schur complement of the
    subdomain's own matrix (Section 2.4), for nodes at every depth, checked
    from the micro-blocks up; floating subdomains have S 1 = 0 and are PSD,
    boundary-touching ones are PD."""
    O = oracle_mod
    kappa = np.random.default_rng(3).uniform(0.2, 5.0, size=(1, n + 1, n + 1, 2))
    f = np.random.default_rng(4).uniform(0.0, 1.0, size=(n + 2, n + 2))
    o = H.hdd_default_opts(n, H.HDD_FP64, leaf=leaf, flags=flags | H.HDD_FLAG_KEEP_FRAMES)
    t = H.HDD(o, 1)
    t.build(kappa, f)
    nc = n + 1
    levels = H.hdd_plan_summary(o)["levels"]
    say("node schur n", n, "levels", levels, "flags", flags, "sync", t.sync(), "last_node", t.last_node())
    errs = []
    for d in range(levels - 1, 0, -1):
        nodes = H.hdd_plan_level(o, d)["nodes"]
        for k in sorted({0, nodes // 2, nodes - 1, min(5, nodes - 1)}):
            info = H.hdd_plan_node(o, d, k)
            S, g, ids = t.node_schur(0, d, k)
            rect = (info["x0"], info["x0"] + info["w"], info["y0"], info["y0"] + info["h"])
            So, go, bnodes = O.subdomain_schur(n, kappa[0], f, rect, drop_dirichlet=(d < levels - 1))
            pos = {(i, j): q for q, (i, j) in enumerate(bnodes)}
            perm = [pos[(int(x) % (nc + 1), int(x) // (nc + 1))] for x in ids]
            So = So[np.ix_(perm, perm)]
            go = go[perm]
            sc = np.abs(So).max()
            eS = np.abs(S - So).max() / sc
            eg = np.abs(g - go).max() / max(np.abs(go).max(), 1e-30)
            say(f"  depth {d} node {k} rect {rect} |Gamma| {len(ids)} errS {eS:.2e} errg {eg:.2e}")
            errs.append((d, k, eS, eg, S, info))
    for d, k, eS, eg, S, info in errs:
        assert eS < 1e-12 and eg < 1e-12, (d, k, eS, eg)
        sc = np.abs(S).max()
        touches = info["x0"] == 0 or info["y0"] == 0 or info["x0"] + info["w"] == nc or info["y0"] + info["h"] == nc
        ev = np.linalg.eigvalsh(S)
        if not touches:
            assert np.abs(S.sum(axis=1)).max() < 1e-12 * sc
            assert ev[0] > -1e-12 * ev[-1]
        elif d < levels - 1:
            assert ev[0] > 0
    assert len(errs) > 3
    t.close()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("n,leaf", [(63, 8), (127, 16)])
def test_node_schur_fp32(H, oracle_mod, n, leaf, fused):
    """The float32 matrix-core levels (fused narrow-interface merges, the fused
    elimination of 63-node interfaces, and the separate panel + Schur-update
    launches that HDD_FLAG_NO_FUSED selects everywhere) produce S_omega and
    g_omega equal to the dense Schur complement of the subdomain's own matrix
    to float32 accuracy."""
    O = oracle_mod
    kappa = np.random.default_rng(5).uniform(0.2, 5.0, size=(1, n + 1, n + 1, 2))
    f = np.random.default_rng(6).uniform(0.0, 1.0, size=(n + 2, n + 2))
    flags = H.HDD_FLAG_KEEP_FRAMES | (0 if fused else H.HDD_FLAG_NO_FUSED)
    o = H.hdd_default_opts(n, H.HDD_FP32_REFINE, leaf=leaf, flags=flags)
    t = H.HDD(o, 1)
    t.build(kappa, f)
    nc = n + 1
    levels = H.hdd_plan_summary(o)["levels"]
    say("fp32 node schur n", n, "levels", levels, "sync", t.sync())
    worst = 0.0
    for d in range(levels - 2, 0, -1):
        nodes = H.hdd_plan_level(o, d)["nodes"]
        for k in sorted({0, nodes // 2, nodes - 1}):
            info = H.hdd_plan_node(o, d, k)
            if (info["w"] - 1) * (info["h"] - 1) > 4000:  # dense brute force stays small
                continue
            S, g, ids = t.node_schur(0, d, k)
            rect = (info["x0"], info["x0"] + info["w"], info["y0"], info["y0"] + info["h"])
            So, go, bnodes = O.subdomain_schur(n, kappa[0], f, rect, drop_dirichlet=True)
            pos = {(i, j): q for q, (i, j) in enumerate(bnodes)}
            perm = [pos[(int(x) % (nc + 1), int(x) // (nc + 1))] for x in ids]
            So = So[np.ix_(perm, perm)]
            go = go[perm]
            eS = np.abs(S - So).max() / np.abs(So).max()
            eg = np.abs(g - go).max() / max(np.abs(go).max(), 1e-30)
            say(f"  depth {d} node {k} gamma {info['gam']} |Gamma| {len(ids)} errS {eS:.2e} errg {eg:.2e}")
            worst = max(worst, eS, eg)
    # float32 frames: a few hundred units of float32 rounding
    assert worst < 5e-5, worst
    t.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_c0_fp32_refine(H, oracle_mod, flags):
    """float32 frames + float64 refinement against the oracle, with matrix
    cores and (flags=1) with the plain FMA updates everywhere, blocks
    included."""
    w = make_workload("c0_63")
    say("c0_63 fp32+refine flags", flags)
    o = H.hdd_default_opts(w.n, H.HDD_FP32_REFINE, leaf=w.leaf, flags=flags)
    t = H.HDD(o, 1)
    t.build(w.kappa, w.f)
    ref = oracle_values(oracle_mod, w.n, w.kappa[0], w.f, w.points)
    got = t.query_points(w.points)[0]
    est, sweeps = t.error_estimate()
    say("fp32 err", rel(got, ref["pts"]), "est", est, "sweeps", sweeps)
    assert rel(got, ref["pts"]) < TOL32
    assert rel(t.query_interface()[0], ref["iface"]) < TOL32
    assert 1 <= sweeps <= o.max_refine
    t.close()


def test_batched_equals_solo(H):
    """Each sample's result is the same alone and inside a batch (bitwise):
    the per-(node, sample) arithmetic does not depend on the batch."""
    w = make_workload("c1_255", n_samples=3)
    say("batched vs solo 255^2")
    for prec in (H.HDD_FP64, H.HDD_FP32_REFINE):
        o = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
        t = H.HDD(o, 3)
        t.build(w.kappa, w.f)
        batch = t.query_points(w.points)
        for s in range(3):
            t.build(w.kappa[s:s + 1], w.f)
            solo = t.query_points(w.points)[0]
            assert np.array_equal(solo, batch[s]), (prec, s)
        t.close()


def test_c1_subset_parity(H, oracle_mod):
    w = make_workload("c1_255", n_samples=2)
    say("c1_255 parity, 2 samples")
    refs = [oracle_values(oracle_mod, w.n, w.kappa[s], w.f, w.points) for s in range(2)]
    for prec, tol in ((H.HDD_FP64, TOL64), (H.HDD_FP32_REFINE, TOL32)):
        o = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
        t = H.HDD(o, 2)
        t.build(w.kappa, w.f)
        got = t.query_points(w.points)
        iface = t.query_interface()
        for s in range(2):
            say(prec, s, rel(got[s], refs[s]["pts"]), rel(iface[s], refs[s]["iface"]))
            assert rel(got[s], refs[s]["pts"]) < tol
            assert rel(iface[s], refs[s]["iface"]) < tol
        t.close()


def test_loglik(H, oracle_mod):
    O = oracle_mod
    w = make_workload("c0_63", n_samples=4)
    say("loglik")
    ut, _ = O.solve(w.n, w.kappa_true[0], w.f)
    y = O.point_values(w.n, ut, w.points) + w.noise
    o = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
    t = H.HDD(o, 4)
    t.build(w.kappa, w.f)
    for normalized in (False, True):
        ll = t.loglik(w.points, y, w.sigma_y, normalized)
        for s in range(4):
            u, _ = O.solve(w.n, w.kappa[s], w.f)
            ref = O.loglik(y, O.point_values(w.n, u, w.points), w.sigma_y, normalized)
            # |d ll| <= sum |r_i| |du_i| / sigma^2 with |du| <= 1e-10 |u|
            bound = np.sum(np.abs(y - O.point_values(w.n, u, w.points))) * 1e-10 * np.abs(u).max() / w.sigma_y ** 2
            assert abs(ll[s] - ref) <= bound + 1e-12 * abs(ref)
    t.close()


def test_invalid_kappa(H):
    w = make_workload("c0_63")
    o = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
    t = H.HDD(o, 1)
    k = w.kappa.copy()
    k[0, 3, 4, 1] = -1.0
    with pytest.raises(H.HddError) as e:
        t.build(k, w.f)
    assert e.value.code == H.HDD_EINVAL
    import torch
    kd = torch.from_numpy(w.kappa.copy()).cuda()
    kd[0, 5, 5, 0] = float("nan")
    fd = torch.from_numpy(w.f).cuda()
    t.build(kd, fd)
    assert t.sync() == H.HDD_EINVAL
    t.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_reused_frames_match_kept_frames(H, prec):
    """Handles that reuse frame memory across levels (the default: only the
    retained factors of every node stay) give the same values, bit for bit,
    as handles that keep every frame, and refuse the frame inspection calls."""
    from workload import make_workload

    w = make_workload("s_255", n_samples=3)
    outs = []
    for flags in (0, H.HDD_FLAG_KEEP_FRAMES):
        o = H.hdd_default_opts(w.n, prec, leaf=w.leaf, flags=flags)
        t = H.HDD(o, 3)
        t.build(w.kappa, w.f)
        outs.append((t.query_points(w.points), t.query_interface(2, 1), t.query_mean([0.25, 0.5, 0.25, 0.5])))
        if flags == 0:
            with pytest.raises(H.HddError) as e:
                t.node_schur(0, 2, 0)
            assert e.value.code == H.HDD_ESTATE
        t.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_large_tile_schur_fp32_vs_fp64(H):
    """The 128 x 128 float32 Schur-update tiles (levels with |gamma| >= 96 and
    at least 192 rows below the interface: the three-workgroup K loop, the
    diagonal tiles' skipped blocks and their load row, the compact tile grid)
    give S_omega and g_omega within float32 rounding of the float64 levels.
    The float64 path is the one certified node by node against the dense
    Schur complement (test_node_schur_bruteforce) and end to end against the
    oracle; the float32 frames are compared with it at 511^2, where the dense
    brute force no longer fits, on the first, middle and last node of every
    level that takes the large tile (measured about 3e-7 for S at 2047^2)."""
    from workload import make_workload

    w = make_workload("s_511", n_samples=1)
    S = {}
    for prec in (H.HDD_FP64, H.HDD_FP32_REFINE):
        o = H.hdd_default_opts(w.n, prec, leaf=w.leaf, flags=H.HDD_FLAG_KEEP_FRAMES)
        t = H.HDD(o, 1)
        t.build(w.kappa, w.f)
        assert t.sync() == 0
        levels = H.hdd_plan_summary(o)["levels"]
        for d in range(levels - 1):
            lv = H.hdd_plan_level(o, d)
            big = lv["gam"] >= 96 and lv["max_U"] + 1 - lv["gam"] >= 192
            if prec == H.HDD_FP32_REFINE and (lv["fp64"] or not big):
                continue
            for k in sorted({0, lv["nodes"] // 2, lv["nodes"] - 1}):
                S[(prec, d, k)] = t.node_schur(0, d, k)[:2]
        t.close()
    checked = 0
    for (prec, d, k), (s32, g32) in S.items():
        if prec != H.HDD_FP32_REFINE:
            continue
        s64, g64 = S[(H.HDD_FP64, d, k)]
        eS = np.abs(s32 - s64).max() / np.abs(s64).max()
        eg = np.abs(g32 - g64).max() / np.abs(g64).max()
        say(f"  depth {d} node {k}: |Gamma| {len(g64)} S {eS:.2e} g {eg:.2e}")
        assert eS < 1e-5 and eg < 1e-4, (d, k, eS, eg)
        checked += 1
    assert checked >= 6
