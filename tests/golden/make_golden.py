"""Write oracle values for the large workloads (calls only oracle/ and workloads/).

For each workload the targets are a seeded subset of the points; the file
stores the target indices and the oracle's u = A q at those targets, all
right-hand sides. Usage:

    python tests/golden/make_golden.py two_layer_hf three_layer
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

SPECS = {
    # name: (workload factory, number of targets, seed of the subset)
    "two_layer_hf": (workloads.two_layer_hf, 2048, 2),
    "three_layer": (workloads.three_layer_ellipses, 1000, 3),
    # the largest geometry of the batched workload, 8 right-hand sides
    "batched_largest": (lambda: workloads.batched_geometry(workloads.BATCHED_LARGEST, nrhs=8), 512, 4),
}


def target_subset(n, m, seed):
    rng = workloads.rng_for(1703, 9136, seed, 999)
    return np.sort(rng.choice(n, size=m, replace=False))


def make(name):
    factory, m, seed = SPECS[name]
    w = factory()
    tid = target_subset(w.n, m, seed)
    t0 = time.time()
    u = oracle.direct_apply(oracle.Media(w.k, w.interfaces), w.xy, w.q, targets=tid)
    dt = time.time() - t0
    path = os.path.join(HERE, name + "_oracle.npz")
    np.savez(path, targets=tid, u=np.atleast_2d(u), seconds=dt, n=w.n,
             workers=len(os.sched_getaffinity(0)))
    print("%s: %d targets, %.1f s -> %s" % (name, m, dt, path), flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(SPECS):
        make(nm)
