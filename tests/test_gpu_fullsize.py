"""Full-size GPU parity against oracle values stored by tests/golden/make_golden.py.

The 255^2 configuration is checked on all 256 samples built in one batch; the
1023^2 configuration on its first 4 samples (points, root midline interface,
mean over [0.25,0.5]^2).  A property that holds at any size certifies the
float64 field at 1023^2: the extended-precision residual bounds its error.
The refined float32 field is compared with that float64 field on every node;
in the 128-sample batch the benchmark times every float64 field is certified
by its residual bound and the float32 path is compared against it.
Tolerances (normwise relative): HDD_FP64 1e-10, HDD_FP32_REFINE 1e-8.
"""
import json
import os
import sys

import numpy as np
import pytest

try:  # import at collection so a slow first import is not charged to a test
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

from workload import make_workload

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-10, 1: 1e-8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gold(name):
    with open(os.path.join(HERE, "golden", f"{name}.json")) as fh:
        return json.load(fh)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_02207_amd import hdd
    return hdd


@pytest.mark.parametrize("prec", [0, 1])
def test_c1_all_256_samples(H, prec):
    g = gold("c1_255")
    w = make_workload("c1_255")
    assert w.kappa.shape[0] == 256
    say("c1_255 all samples, precision", prec)
    o = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
    t = H.HDD(o, 256)
    t.build(torch.from_numpy(w.kappa).cuda(), torch.from_numpy(w.f).cuda())
    pts = t.query_points(np.array(g["points"]))
    worst = max(rel(pts[s["sample"]], s["points"]) for s in g["samples"])
    say("  worst rel err over 256 samples", worst)
    assert worst < TOL[prec]
    ll = t.loglik(np.array(g["points"]), np.array(g["y"]), g["sigma_y"])
    for s in g["samples"][:8]:
        r = np.array(g["y"]) - np.array(s["points"])
        ref = -float(r @ r) / (2 * g["sigma_y"] ** 2)
        bound = np.abs(r).sum() * TOL[prec] * np.abs(s["points"]).max() / g["sigma_y"] ** 2
        assert abs(ll[s["sample"]] - ref) <= bound + 1e-12 * abs(ref)
    t.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_1023(H, oracle_mod, prec):
    g = gold("c2_1023")
    w = make_workload("c2_1023")
    ns = len(g["samples"])
    say("c2_1023 precision", prec, "samples", ns)
    o = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
    t = H.HDD(o, ns)
    kd = torch.from_numpy(w.kappa[:ns]).cuda()
    fd = torch.from_numpy(w.f).cuda()
    t.build(kd, fd)
    pts = t.query_points(np.array(g["points"]))
    iface = t.query_interface()
    mean = t.query_mean(g["mean_rect"])
    for s in g["samples"]:
        k = s["sample"]
        e = (rel(pts[k], s["points"]), rel(iface[k], s["interface"]), rel([mean[k]], [s["mean"]]))
        say(f"  sample {k}: points {e[0]:.2e} interface {e[1]:.2e} mean {e[2]:.2e}")
        assert max(e) < TOL[prec]
    est, sweeps = t.error_estimate()
    say("  refinement sweeps", sweeps, "estimate", est)
    t.solve_full()
    u = t.solution(0)
    if prec == 0:
        # property at any size: ||u - u_h||_2 <= ||b - A u||_2 / lambda_min(A)
        # (rigorous; pessimistic by kappa_max / kappa_min and the spectrum)
        r = oracle_mod.residual(w.n, w.kappa[0], w.f, u)
        bound = oracle_mod.error_bound_l2(w.n, w.kappa[0], r)
        say("  residual error bound (l2)", bound, "field norm", np.linalg.norm(u))
        assert bound <= 1e-8 * np.linalg.norm(u)
    else:
        # the whole refined field against the float64 path (certified above
        # by the residual bound) on every node
        o64 = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
        t64 = H.HDD(o64, 1)
        t64.build(kd[:1].contiguous(), fd)
        t64.solve_full()
        u64 = t64.solution(0)
        t64.close()
        e = rel(u, u64)
        say("  field vs float64 path (max norm)", e)
        assert e < TOL[prec]
    t.close()


@pytest.mark.parametrize("variant", ["no_fused", "all_float32"])
def test_c2_1023_variants(H, variant):
    """The same stored oracle values at 1023^2 from the separate extend-add,
    panel and Schur-update launches on every level (HDD_FLAG_NO_FUSED, the
    cross-check of the fused merges), and with every level in float32
    (fp64_top_levels = 0, the variant the benchmark reports beside the
    headline)."""
    g = gold("c2_1023")
    w = make_workload("c2_1023")
    ns = len(g["samples"])
    say("c2_1023 variant", variant)
    o = H.hdd_default_opts(w.n, H.HDD_FP32_REFINE, leaf=w.leaf)
    if variant == "no_fused":
        o.flags = H.HDD_FLAG_NO_FUSED
    else:
        o.fp64_top_levels = 0
    t = H.HDD(o, ns)
    t.build(torch.from_numpy(w.kappa[:ns]).cuda(), torch.from_numpy(w.f).cuda())
    pts = t.query_points(np.array(g["points"]))
    iface = t.query_interface()
    mean = t.query_mean(g["mean_rect"])
    for s in g["samples"]:
        k = s["sample"]
        e = (rel(pts[k], s["points"]), rel(iface[k], s["interface"]), rel([mean[k]], [s["mean"]]))
        say(f"  sample {k}: points {e[0]:.2e} interface {e[1]:.2e} mean {e[2]:.2e}")
        assert max(e) < TOL[1]
    est, sweeps = t.error_estimate()
    say("  refinement sweeps", sweeps)
    t.close()


def test_c2_1023_bench_batch(H, oracle_mod):
    """The bench's launch configuration (128 samples of the 1023^2 workload
    in one batch, default options).  Every sample's float64 field is certified
    against the exact discrete solution by its extended-precision residual
    bound (a property that holds at any size: ||u - u_h||_2 <= ||b - A u||_2 /
    lambda_min(A)); every sample's measurements on the FP32 matrix-core +
    refinement path agree with that certified float64 path to 1e-8, and the
    first 4 samples with the stored oracle values."""
    g = gold("c2_1023")
    B = 128
    w = make_workload("c2_1023", n_samples=B)
    kd = torch.from_numpy(w.kappa).cuda()
    fd = torch.from_numpy(w.f).cuda()
    xy = np.array(g["points"])
    out = {}
    for prec in (H.HDD_FP64, H.HDD_FP32_REFINE):
        say("c2_1023 batch", B, "precision", prec)
        t = H.HDD(H.hdd_default_opts(w.n, prec, leaf=w.leaf), B)
        t.build(kd, fd)
        out[prec] = (t.query_points(xy), t.query_interface(), t.query_mean(g["mean_rect"]))
        if prec == H.HDD_FP32_REFINE:
            say("  refinement sweeps", t.error_estimate()[1])
        else:
            t.solve_full()
            worst_b = 0.0
            for s in range(B):
                u = t.solution(s)
                r = oracle_mod.residual(w.n, w.kappa[s], w.f, u)
                b = oracle_mod.error_bound_l2(w.n, w.kappa[s], r) / np.linalg.norm(u)
                worst_b = max(worst_b, b)
                assert b <= 1e-8, (s, b)
            say("  float64 fields: worst certified relative l2 error bound over", B, "samples", worst_b)
        t.close()
    worst = 0.0
    for s in range(B):
        for a, b in zip(out[H.HDD_FP32_REFINE], out[H.HDD_FP64]):
            worst = max(worst, rel(np.atleast_1d(a[s]), np.atleast_1d(b[s])))
    say("  worst rel difference over", B, "samples", worst)
    assert worst < TOL[1]
    for smp in g["samples"]:
        k = smp["sample"]
        for prec in (H.HDD_FP64, H.HDD_FP32_REFINE):
            assert rel(out[prec][0][k], smp["points"]) < TOL[prec]
            assert rel(out[prec][1][k], smp["interface"]) < TOL[prec]


def test_c4_2047_stress(H, oracle_mod):
    """High-contrast stress workload (2047^2 interior nodes, kappa variance 4,
    correlation length 0.02, 200 modes, Gaussian-bump load).  The oracle's
    banded solve does not fit a test here, so parity with it is unpinned at
    this size; instead the float64 field is certified by its
    extended-precision residual bound, which carries kappa_max / kappa_min
    (about 1e4 here) and h^-2 and was measured at 8.5e-8 relative (gate
    1e-6).  The float32 matrix-core + refinement path matches that float64
    field to 1e-8 (measured 1.6e-10)."""
    w = make_workload("c4_2047")
    xy = np.asarray(w.points)
    kd = torch.from_numpy(w.kappa[:1]).cuda()
    fd = torch.from_numpy(w.f).cuda()
    say("c4_2047 kappa range", float(w.kappa.min()), float(w.kappa.max()))
    out = {}
    for prec in (H.HDD_FP64, H.HDD_FP32_REFINE):
        t = H.HDD(H.hdd_default_opts(w.n, prec, leaf=w.leaf), 1)
        t.build(kd, fd)
        pts = t.query_points(xy)[0]
        iface = t.query_interface()[0]
        est, sweeps = t.error_estimate()
        t.solve_full()
        u = t.solution(0)
        out[prec] = (pts, iface, u)
        say("  precision", prec, "sweeps", sweeps, "estimate", est)
        t.close()
    r = oracle_mod.residual(w.n, w.kappa[0], w.f, out[H.HDD_FP64][2])
    bound = oracle_mod.error_bound_l2(w.n, w.kappa[0], r)
    say("  float64 residual error bound (l2)", bound, "field norm", np.linalg.norm(out[H.HDD_FP64][2]))
    assert bound <= 1e-6 * np.linalg.norm(out[H.HDD_FP64][2])
    e = max(rel(out[H.HDD_FP32_REFINE][0], out[H.HDD_FP64][0]), rel(out[H.HDD_FP32_REFINE][1], out[H.HDD_FP64][1]),
            rel(out[H.HDD_FP32_REFINE][2], out[H.HDD_FP64][2]))
    say("  float32+refinement vs float64 (max over points, midline, field)", e)
    assert e < 1e-8
