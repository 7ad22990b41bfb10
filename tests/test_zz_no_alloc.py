"""hdd_create_static (workspace in the library's static device array, no
allocation) against hdd_create on the same inputs, and both against the
oracle: two handles in a row on the same array, the second for a smaller
mesh and batch, in both precision modes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _outputs(H, opts, ns, kappa, f, pts, y, sigma, workspace):
    t = H.HDD(opts, ns, workspace=workspace)
    try:
        t.build(kappa, f)
        u = t.query_points(pts)
        ll = t.loglik(pts, y, sigma)
        mid = t.query_interface(0, 0)
        mean = t.query_mean([0.25, 0.5, 0.25, 0.5])
        status = t.sample_status()
    finally:
        t.close()
    return u, ll, mid, mean, status


@pytest.mark.parametrize("precision", [0, 1])
def test_static_workspace_matches_hdd_create(precision, oracle_mod):
    import torch

    from paper_1708_02207_amd import hdd as H
    from workload.gen import coefficient_field, rhs_nodal

    O = oracle_mod
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    tol = 1e-10 if precision == H.HDD_FP64 else 1e-8
    # first call: 63^2 with 4 samples; second: 31^2 with 2 samples (smaller
    # input on the same static array, which keeps the first call's contents)
    for n, ns, seed in ((63, 4, 11), (31, 2, 12)):
        opts = H.hdd_default_opts(n, precision, leaf=8)
        assert H.hdd_workspace_size(opts, ns) <= H.STATIC_WORKSPACE_BYTES
        rng = np.random.default_rng(seed)
        z = rng.standard_normal((ns, 10))
        pts = rng.uniform(size=(8, 2))
        kappa = np.ascontiguousarray(coefficient_field(n, z, 0.5, 0.2))
        f = rhs_nodal(n, "one")
        y = np.full(len(pts), 0.01)
        print(f"static workspace: n={n} samples={ns} precision={precision}", flush=True)
        ref = _outputs(H, opts, ns, kappa, f, pts, y, 0.01, "torch")
        got = _outputs(H, opts, ns, kappa, f, pts, y, 0.01, "static")
        for a, b in zip(ref[:4], got[:4]):
            a, b = np.asarray(a), np.asarray(b)
            assert np.abs(a - b).max() <= 1e-12 * max(np.abs(a).max(), 1e-300)
        assert (got[4] == 0).all()
        # both against the oracle
        for s in range(ns):
            u_ref, _ = O.solve(n, kappa[s], f)
            pv = O.point_values(n, u_ref, pts)
            assert np.abs(got[0][s] - pv).max() <= tol * np.abs(pv).max()
            mid = O.interface_values(n, u_ref)
            assert np.abs(got[2][s] - mid).max() <= tol * np.abs(mid).max()


def test_static_workspace_limits():
    import torch

    from paper_1708_02207_amd import hdd as H

    torch.cuda.set_device(0)
    big = H.hdd_default_opts(511, H.HDD_FP64)
    assert H.hdd_workspace_size(big, 1) > H.STATIC_WORKSPACE_BYTES
    with pytest.raises(H.HddError) as e:
        H.HDD(big, 1, workspace="static")
    assert e.value.code == H.HDD_ENOMEM
    small = H.hdd_default_opts(31, H.HDD_FP64)
    a = H.HDD(small, 1, workspace="static")
    try:
        with pytest.raises(H.HddError) as e:
            H.HDD(small, 1, workspace="static")  # one live static handle per GPU
        assert e.value.code == H.HDD_ESTATE
        with pytest.raises(H.HddError) as e:
            a.timing_enable(1)
        assert e.value.code == H.HDD_EINVAL
    finally:
        a.close()
    b = H.HDD(small, 1, workspace="static")  # released by hdd_destroy
    b.close()
