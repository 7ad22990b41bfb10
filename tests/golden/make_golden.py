"""Write the stored expected values of the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generator
(workload/); nothing here touches the GPU library.  For each configuration
it stores the oracle's query values for the first samples of the seeded
batch and the synthetic observations y = u_true(sites) + noise, where u_true
is the oracle solution for the configuration's Z_true.

Usage: python tests/golden/make_golden.py [c0_63 c1_255 c2_1023] [--jobs J]
The 1023^2 solves take several minutes each and about 9 GB of memory.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workload import make_workload  # noqa: E402

PLAN = {
    "c0_63": dict(samples=4),
    "c1_255": dict(samples=256),
    "c2_1023": dict(samples=4),
}


def _digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def _solve_one(args):
    name, s, true = args
    w = make_workload(name, n_samples=PLAN[name]["samples"])
    kap = w.kappa_true[0] if true else w.kappa[s]
    t0 = time.time()
    u, rr = O.solve(w.n, kap, w.f)
    out = dict(sample=s, true=true, relres=rr, seconds=time.time() - t0,
               points=O.point_values(w.n, u, w.points).tolist(), kappa_sha=_digest(kap))
    if w.interface:
        out["interface"] = O.interface_values(w.n, u).tolist()
    if w.mean_rect is not None:
        out["mean"] = O.mean_value(w.n, u, w.mean_rect)
    return out


def make(name: str, jobs: int):
    w = make_workload(name, n_samples=PLAN[name]["samples"])
    tasks = [(name, -1, True)] + [(name, s, False) for s in range(PLAN[name]["samples"])]
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_solve_one, tasks))
    true = res[0]
    y = (np.array(true["points"]) + w.noise).tolist()
    doc = dict(
        config=name, n=w.n, leaf=w.leaf, spec=w.spec, sigma_y=w.sigma_y,
        points=w.points.tolist(), y=y, mean_rect=w.mean_rect,
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
