"""Write the stored expected values of the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generator
(workload/); nothing here touches the GPU library.  For each configuration
it stores the oracle's query values for the first samples of the seeded
batch and the synthetic observations y = u_true(sites) + noise, where u_true
is the oracle solution for the configuration's Z_true.

Besides the workload's own outputs, each sample stores the values at the
edge-case sites of workload.edge_sites, u on the interfaces of a few tree
nodes (oracle.node_interface) and the means over the rectangles of
workload.off_tree_rects, which are not tree nodes.

Usage: python tests/golden/make_golden.py [c0_63 c1_255 s_511 c2_1023] [--jobs J]
The 1023^2 solves take several minutes each and about 9 GB of memory.
"""
from __future__ import annotations

import os

# one BLAS thread per worker process (the workers run in parallel)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workload import edge_sites, make_workload, off_tree_rects  # noqa: E402

PLAN = {
    "c0_63": dict(samples=4),
    "c1_255": dict(samples=256),
    "s_511": dict(samples=4),
    "c2_1023": dict(samples=4),
}
# tree nodes (index in the oracle's tree_rects order, blocks of 16 x 16 cells
# or of the leaf size if smaller) whose interface values are stored
NODES = {
    "c0_63": [0, 1, 2, 5, 12, 27, 62],
    "c1_255": [0, 1, 2, 5, 12, 27, 60, 130, 254],
    "s_511": [0, 1, 2, 5, 12, 27, 60, 130, 300, 700, 1022],
    "c2_1023": [0, 1, 2, 6, 13, 30, 63, 130, 260, 600, 1300, 2600, 4094],
}


def _digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


_WORKLOADS = {}


def _workload(name):
    if name not in _WORKLOADS:
        _WORKLOADS[name] = make_workload(name, n_samples=PLAN[name]["samples"])
    return _WORKLOADS[name]


def _solve_one(args):
    name, s, true = args
    w = _workload(name)
    kap = w.kappa_true[0] if true else w.kappa[s]
    t0 = time.time()
    u, rr = O.solve(w.n, kap, w.f)
    out = dict(sample=s, true=true, relres=rr, seconds=time.time() - t0,
               points=O.point_values(w.n, u, w.points).tolist(), kappa_sha=_digest(kap))
    if w.interface:
        out["interface"] = O.interface_values(w.n, u).tolist()
    if w.mean_rect is not None:
        out["mean"] = O.mean_value(w.n, u, w.mean_rect)
    # edge-case sites, interfaces of inner tree nodes, means over rectangles
    # that are not tree nodes (samples only: the true field feeds y alone)
    if not true and (name != "c1_255" or s < 8):
        out["edge_points"] = O.point_values(w.n, u, edge_sites(w.n)).tolist()
        block = min(16, w.leaf)
        out["node_interfaces"] = {str(k): O.node_interface(w.n, u, block, k)[1].tolist() for k in NODES[name]}
        out["off_tree_means"] = [O.mean_value(w.n, u, r) for r in off_tree_rects(w.n)]
    return out


def make(name: str, jobs: int):
    w = make_workload(name, n_samples=PLAN[name]["samples"])
    tasks = [(name, -1, True)] + [(name, s, False) for s in range(PLAN[name]["samples"])]
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_solve_one, tasks))
    true = res[0]
    y = (np.array(true["points"]) + w.noise).tolist()
    block = min(16, w.leaf)
    doc = dict(
        config=name, n=w.n, leaf=w.leaf, spec=w.spec, sigma_y=w.sigma_y,
        points=w.points.tolist(), y=y, mean_rect=w.mean_rect,
        edge_sites=edge_sites(w.n).tolist(), off_tree_rects=[list(r) for r in off_tree_rects(w.n)],
        interface_block=block,
        node_interface_ids={str(k): O.node_interface(w.n, np.zeros((w.n + 2, w.n + 2)), block, k)[0].tolist()
                            for k in NODES[name]},
        generator="workload.make_workload", oracle="oracle.solve (banded Cholesky + 2 extended-precision sweeps)",
        samples=res[1:], true=true,
    )
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path}: {len(res) - 1} samples, worst relres {max(r['relres'] for r in res):.2e}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="*", default=list(PLAN))
    ap.add_argument("--jobs", type=int, default=2)
    a = ap.parse_args()
    for c in a.configs:
        make(c, a.jobs)
