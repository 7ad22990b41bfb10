"""Captured launch sequences and the tile autotuner.

The build, the first full Root to Leaves and every refinement sweep are
replayed from HIP graphs captured once per sample count.  A handle replaying
graphs must give exactly the values of a handle that issues every launch
eagerly (HDD_FLAG_NO_GRAPH), on every replay, with eager work (queries,
synchronizations) between the replays and with the sample count changing
between builds.  The autotuner's per-level tile choices must keep the
results at the oracle tolerances.
"""
import numpy as np
import pytest

from workload import make_workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-8}


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1708_02207_amd import hdd
    return hdd


def say(*a):
    print(*a, flush=True)


def _outputs(t, w):
    return (t.query_points(w.points), t.query_interface(1, 1), t.query_mean([0.25, 0.5, 0.25, 0.5]),
            t.loglik(w.points, np.zeros(len(w.points)), 0.01))


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_equal_eager(H, prec):
    w = make_workload("s_255", n_samples=6)
    o_g = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
    o_e = H.hdd_default_opts(w.n, prec, leaf=w.leaf, flags=H.HDD_FLAG_NO_GRAPH)
    tg, te = H.HDD(o_g, 4), H.HDD(o_e, 4)
    # sample counts change between builds: 3, 2, 3 (a cached graph), 4
    for rep, (a, b) in enumerate([(0, 3), (3, 5), (1, 4), (2, 6)]):
        kap = np.ascontiguousarray(w.kappa[a:b])
        say(f"graph replay {rep}: precision {prec}, samples {b - a}")
        tg.build(kap, w.f)
        te.build(kap, w.f)
        og, oe = _outputs(tg, w), _outputs(te, w)
        for x, y in zip(og, oe):
            assert np.array_equal(x, y), rep
        assert tg.sync() == 0 and te.sync() == 0
    gi, ge = tg.graph_info(), te.graph_info()
    say("graph nodes", gi, "eager handle", ge)
    assert gi["build_nodes"] > 0 and gi["launches"] > 0
    if prec == 1:  # float32 + refinement solves the full field: both sweep graphs exist
        assert gi["solve_nodes"] > 0 and gi["sweep_nodes"] > 0
    assert ge["launches"] == 0 and ge["build_nodes"] == 0
    tg.close()
    te.close()


def test_graph_replay_solve_rhs(H, oracle_mod):
    """Further loads through the replayed sweep graph equal the eager sweeps."""
    w = make_workload("s_127", n_samples=2)
    f2 = np.random.default_rng(5).uniform(0.0, 1.0, size=w.f.shape)
    res = []
    for flags in (0, H.HDD_FLAG_NO_GRAPH):
        t = H.HDD(H.hdd_default_opts(w.n, 1, leaf=w.leaf, flags=flags), 2)
        t.build(w.kappa, w.f)
        vals = []
        for _ in range(3):
            t.solve_rhs(f2)
            vals.append(t.solution(1))
        res.append(vals)
        t.close()
    for x, y in zip(*res):
        assert np.array_equal(x, y)
    u_ref, _ = oracle_mod.solve(w.n, w.kappa[1], f2)
    assert np.abs(res[0][-1] - u_ref).max() <= TOL[1] * np.abs(u_ref).max()


@pytest.mark.parametrize("name", ["s_511", "c2_1023"])
def test_autotune_keeps_parity(H, oracle_mod, name):
    """Tile choices from the autotuner (timed on this GPU) leave the float32 +
    refinement results within 1e-8 of the float64 path certified against the
    oracle (stored oracle values at 1023^2, a live oracle solve at 511^2)."""
    import json
    import os

    ns = 2
    w = make_workload(name, n_samples=ns)
    t = H.HDD(H.hdd_default_opts(w.n, 1, leaf=w.leaf), ns)
    t.build(w.kappa, w.f)
    ch = t.autotune(1)
    say(f"{name}: tile choices per level {ch.tolist()}")
    assert set(ch.tolist()) <= {0, 64, 128} and (ch > 0).any()
    pts = t.query_points(w.points)
    t.build(w.kappa, w.f)  # a later build replays with the chosen tiles
    pts2 = t.query_points(w.points)
    t.close()
    assert np.array_equal(pts, pts2)
    path = os.path.join(os.path.dirname(__file__), "golden", f"{name}.json")
    g = json.load(open(path))
    for smp in g["samples"][:ns]:
        s = smp["sample"]
        ref = np.array(smp["points"])
        xy = np.array(g["points"])
        assert np.allclose(xy, w.points)
        e = np.abs(pts[s] - ref).max() / np.abs(ref).max()
        say(f"  sample {s}: rel err {e:.2e}")
        assert e < TOL[1]
