"""Sample-specific queries and the continuous-batching server, against the
oracle (normwise relative tolerances: HDD_FP32_REFINE 1e-8)."""
import sys
import threading

import numpy as np
import pytest

try:  # import at collection so a slow first import is not charged to a test
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

from workload import make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def test_ragged_queries(H):
    """Each sample's own sites give the values the uniform query gives for
    those sites, and the per-sample log-likelihood equals its closed form."""
    w = make_workload("s_127", n_samples=6)
    rng = np.random.default_rng(11)
    t = H.HDD(H.hdd_default_opts(w.n, H.HDD_FP32_REFINE, leaf=w.leaf), 6)
    t.build(w.kappa, w.f)
    sets = [rng.uniform(size=(k, 2)) for k in (1, 7, 32, 3, 16, 5)]
    got = t.query_points_ragged(sets)
    for s, xy in enumerate(sets):
        ref = t.query_points(xy)[s]
        assert np.array_equal(got[s], ref), s
    ys = [v + 0.01 * rng.standard_normal(len(v)) for v in got]
    sig = np.array([0.01, 0.02, 0.01, 0.05, 0.01, 0.03])
    ll = t.loglik_ragged(sets, ys, sig)
    for s in range(6):
        r = ys[s] - got[s]
        assert abs(ll[s] - (-(r @ r) / (2 * sig[s] ** 2))) <= 1e-12 * abs(ll[s]) + 1e-12
    t.close()


def test_server_alone_and_in_the_mix(H, oracle_mod):
    """A request answered alone and the same request answered inside a mix of
    concurrent requests on two mesh sizes both match the oracle to 1e-8; the
    mix is served in fewer batches than requests (continuous batching)."""
    meshes = ["s_127", "c0_63"]
    W = {m: make_workload(m, n_samples=6) for m in meshes}
    srv = H.Server([W[m].n for m in meshes], H.HDD_FP32_REFINE, slots=8, leaves=[W[m].leaf for m in meshes],
                   f=[W[m].f for m in meshes])
    rng = np.random.default_rng(12)
    probe_xy = rng.uniform(size=(9, 2))
    w0 = W["s_127"]
    ref_u, _ = oracle_mod.solve(w0.n, w0.kappa[0], w0.f)
    ref = oracle_mod.point_values(w0.n, ref_u, probe_xy)
    y = ref + 0.01 * rng.standard_normal(len(ref))

    rid = srv.submit(0, w0.kappa[0], probe_xy, y, 0.01)
    alone, ll_alone, tm = srv.result(rid, len(probe_xy))
    say("alone: err", rel(alone, ref), "batch", tm[3])
    assert rel(alone, ref) < TOL

    ids, lock = [], threading.Lock()

    def client(k):
        r = np.random.default_rng(100 + k)
        for j in range(6):
            m = int(r.integers(0, 2))
            w = W[meshes[m]]
            xy = r.uniform(size=(int(r.integers(1, 33)), 2))
            i = srv.submit(m, w.kappa[int(r.integers(0, 6))], xy)
            with lock:
                ids.append((i, len(xy)))

    threads = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    rid = srv.submit(0, w0.kappa[0], probe_xy, y, 0.01)
    for th in threads:
        th.join()
    mixed, ll_mixed, tm = srv.result(rid, len(probe_xy))
    for i, n in ids:
        srv.result(i, n)
    st = srv.stats()
    say("mixed: err", rel(mixed, ref), "batch", tm[3], "stats", st)
    assert rel(mixed, ref) < TOL
    assert rel(mixed, alone) < 2 * TOL
    r = y - mixed
    assert abs(ll_mixed - (-(r @ r) / (2 * 0.01 ** 2))) <= 1e-9 * abs(ll_mixed)
    assert abs(ll_mixed - ll_alone) <= np.abs(r).sum() * 2 * TOL * np.abs(ref).max() / 0.01 ** 2 + 1e-9
    assert st["completed"] == st["submitted"] == len(ids) + 2
    assert st["batches"] < st["completed"]
    srv.close()
