"""Input generator: determinism, shapes and the stated coefficient model."""
import numpy as np

from workload import CONFIGS, kl_modes, make_workload, paper_kappa, rhs_nodal


def test_deterministic_and_shapes():
    a = make_workload("c0_63")
    b = make_workload("c0_63")
    assert a.kappa.shape == (1, 64, 64, 2) and a.f.shape == (65, 65)
    assert np.array_equal(a.kappa, b.kappa) and np.array_equal(a.points, b.points)
    assert a.points.shape == (5, 2) and (a.kappa > 0).all()


def test_sites_independent_of_batch():
    a = make_workload("c1_255", n_samples=4)
    b = make_workload("c1_255", n_samples=300)
    assert np.array_equal(a.points, b.points)
    assert np.array_equal(a.z, b.z[:4]) and b.z.shape == (300, 20)


def test_modes_ordered_and_q_zero_on_boundary():
    j, k, lam = kl_modes(20, 1.0, 0.1)
    key = j * j + k * k
    assert (np.diff(key) >= 0).all() and (np.diff(lam) <= 0).all()
    assert len(j) == 20


def test_paper_coefficients():
    k = paper_kappa(127, "sin50")
    assert k.shape == (1, 128, 128, 2) and 0.5 <= k.min() and k.max() <= 1.5
    a = paper_kappa(255, "alpha500")
    assert (a > 0).all()
    f = rhs_nodal(63, "bump")
    assert abs(f.max() - 1.0) < 0.05


def test_configs_tree_compatible():
    for name, spec in CONFIGS.items():
        nc = spec["n"] + 1
        ratio = nc // spec["leaf"]
        assert nc % spec["leaf"] == 0 and ratio & (ratio - 1) == 0, name
