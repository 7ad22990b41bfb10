"""u_h on a coarse mesh of interfaces (setup (c) of Fig. HDDidea; Section
3.5): the fine solution on every interface above a depth, from a Root to
Leaves that stops at that depth.  Values against the oracle's field at the
same nodes (live at 255^2, stored interfaces at 1023^2), in both precision
modes; in float64 only the levels above the depth are solved."""
import json
import os

import numpy as np
import pytest

from workload import make_workload

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-10, 1: 1e-8}
KIND_TOPDOWN = 4


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_1708_02207_amd import hdd
    return hdd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def skeleton_ids(H, o, depth):
    ids = []
    for d in range(depth):
        for k in range(H.hdd_plan_level(o, d)["nodes"]):
            info = H.hdd_plan_node(o, d, k)
            ids.extend(info["ids"][: info["gam"]].tolist())
    return np.array(ids)


@pytest.mark.parametrize("prec", [0, 1])
def test_skeleton_against_oracle(H, oracle_mod, prec):
    O = oracle_mod
    w = make_workload("s_255", n_samples=2)
    o = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
    t = H.HDD(o, 2)
    t.build(w.kappa, w.f)
    levels = H.hdd_plan_summary(o)["levels"]
    refs = [O.solve(w.n, w.kappa[s], w.f)[0] for s in range(2)]
    for depth in (1, 3, 5, levels - 1):
        if prec == 0:
            t.timing_enable(1 << KIND_TOPDOWN)
        got = t.query_skeleton(depth)
        if prec == 0:
            per_level = [t.timing_get(KIND_TOPDOWN, level=L)[1] for L in range(levels)]
            t.timing_enable(0)
            say(f"  depth {depth}: top-down launches per level {per_level}")
            assert all(per_level[L] == 0 for L in range(depth, levels))
        ids = skeleton_ids(H, o, depth)
        nc1 = w.n + 2
        for s in range(2):
            ref = refs[s].reshape(-1)[ids]
            e = rel(got[s], ref)
            say(f"skeleton precision {prec} depth {depth} sample {s}: {len(ids)} nodes, rel err {e:.2e}")
            assert e < TOL[prec]
        assert nc1 > 0
    t.close()


def test_skeleton_1023_stored(H):
    """1023^2 in float64: the skeleton above depth 4 contains the interfaces
    of tree nodes 0, 1, 2, 6 and 13 whose oracle values are stored."""
    g = json.load(open(os.path.join(HERE, "golden", "c2_1023.json")))
    ns = 2
    w = make_workload("c2_1023", n_samples=ns)
    o = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
    t = H.HDD(o, ns)
    t.build(w.kappa, w.f)
    depth = 4
    got = t.query_skeleton(depth)
    t.close()
    ids = skeleton_ids(H, o, depth)
    pos = {int(q): p for p, q in enumerate(ids)}
    checked = 0
    for key, nid in g["node_interface_ids"].items():
        nid = [int(q) for q in nid]
        if not all(q in pos for q in nid):
            continue
        for smp in g["samples"][:ns]:
            s = smp["sample"]
            e = rel(got[s][[pos[q] for q in nid]], smp["node_interfaces"][key])
            say(f"  node {key} sample {s}: rel err {e:.2e}")
            assert e < TOL[0]
            checked += 1
    assert checked >= 8
