"""Write oracle reference values for the full-size workloads.

Calls only the FP64 oracle (``oracle/``) on the seeded instances of
``paper_2405_14060_amd.workloads``; the GPU tests compare against the files
written here.  Run from the repository root:  python tests/golden/make_oracle_refs.py
"""
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2405_14060_amd import workloads as W  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def grid20_marginals(seed=0):
    net = W.grid_mrf(20, 20, seed)
    lv = oracle.build_leaves(net)
    pairs = oracle.elimination_tree(lv.labels, lv.card, list(range(net.n_vars)))
    t = time.time()
    lz, marg, *_ = oracle.marginals(net, pairs=pairs)
    ref = dict(workload="grid20x20_mrf", seed=seed, log_z=lz,
               p1=[float(m[1]) for m in marg], oracle_seconds=time.time() - t,
               note="FP64 oracle, bucket-elimination tree in variable-id order")
    with open(os.path.join(OUT, "oracle_grid20x20_seed%d.json" % seed), "w") as f:
        json.dump(ref, f, indent=1)
    print("grid20x20 seed", seed, "log Z", lz)


if __name__ == "__main__":
    grid20_marginals(0)
