#!/usr/bin/env python
"""Benchmark of the hot path: log Z + all single-variable marginals.

Workload: the 20x20 binary grid MRF (400 variables, 400 unary + 760 pairwise
Gaussian log-potential tables, seed 0), contracted along the library's
planned tree (bucket elimination, largest intermediate 2^20 elements).  One
step = one call of tn_marginals: leaf preparation, the forward sum-product
over the tree, the reverse pass (two adjoint contractions per node) and the
marginal normalisation, results copied back to the host.  Factor tables are
resident in device memory before the timed region.

Prints one JSON line; see the design doc for the meaning of every field.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TN-contraction TFLOP/s; logZ+marginal solves/s vs FP64 path at err<=1e-5"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
KIND_NAMES = {0: "contract_map_sum", 1: "contract_map_max", 2: "contract_split_sum",
              3: "contract_split_max", 4: "prepare", 5: "other", 6: "seg_carrier_fwd",
              7: "seg_carrier_bwd", 8: "seg_maps", 9: "seg_adjoint_sweeps", 10: "contract_mfma_sum"}


def kernel_summary(prof):
    names = KIND_NAMES
    agg = {}
    for kind, fl, by, ms in prof:
        a = agg.setdefault(names[kind], dict(n=0, flops=0.0, bytes=0.0, ms=0.0))
        a["n"] += 1
        a["flops"] += fl
        a["bytes"] += by
        a["ms"] += ms
    return agg


def cpu_baseline(net, budget_s=40.0):
    """The FP64 oracle on one solve of the same workload (log Z + marginals)."""
    import oracle
    lv = oracle.build_leaves(net)
    pairs = oracle.elimination_tree(lv.labels, lv.card, list(range(net.n_vars)))
    t0 = time.perf_counter()
    lz, marg, *_ = oracle.marginals(net, pairs=pairs)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="solves/s", cores=1, kind="oracle",
                sample="one full solve (log Z + all 400 marginals) of the same 20x20 grid, "
                       "single-threaded FP64 loop nests, %.1f s" % dt), lz, marg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on more than one GPU are not part of this build "
              "(the path shards by evidence instance or slice, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2405_14060_amd as T
    from paper_2405_14060_amd import workloads as W

    torch.cuda.set_device(0)
    net = W.grid_mrf(20, 20, 0)
    plan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, use_graph=not args.no_graph)
    info = plan.info()

    for _ in range(args.warmup):
        plan.marginals()
    plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lz, m = plan.marginals()
    plan.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    solves_per_s = args.steps / dt

    # per-launch times (HIP events on the plan's stream) for the roofline
    prof = plan.profile(1, reps=3)
    agg = kernel_summary(prof)
    flops_solve = sum(fl for _, fl, _, _ in prof)
    dom_name, dom = max(agg.items(), key=lambda kv: kv[1]["ms"])
    kind_of = {v: k for k, v in KIND_NAMES.items()}
    # the dominant kernel's launches timed back to back between two events
    avg_ms, fl_launch, by_launch, n_launch = plan.profile_kind(1, kind_of[dom_name], reps=5)
    achieved_gbs = by_launch / (avg_ms * 1e-3) / 1e9
    achieved_tf = fl_launch / (avg_ms * 1e-3) / 1e12
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    mfma_frac = achieved_tf / FP32_PEAK_TFLOPS
    if hbm_frac >= mfma_frac:
        roof = dict(bound="hbm", achieved=round(achieved_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(hbm_frac, 4), traffic=None)
    else:
        roof = dict(bound="mfma", achieved=round(achieved_tf, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(mfma_frac, 4), traffic=None)
    roof["kernel"] = dom_name
    roof["launches_per_solve"] = n_launch
    roof["avg_launch_us"] = round(avg_ms * 1e3, 3)
    roof["bytes_per_launch"] = round(by_launch)
    roof["flops_per_launch"] = round(fl_launch)

    out = dict(metric=METRIC, value=round(solves_per_s, 3), unit="solves/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 4),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="grid20x20_mrf logZ+all-marginals", seed=0, n_vars=400,
                           n_factors=1160, tree_sc_log2=info["sc"], tree_tc_log2=round(info["tc"], 3),
                           kernels_per_solve=len(prof),
                           launches_per_solve=info["n_launches_fwd"] + info["n_launches_bwd"] + 3,
                           graph=not args.no_graph),
               tflops=round(flops_solve / (ms_per_step * 1e-3) / 1e12, 4),
               log_z=float(lz[0]), roofline=roof,
               kernels={k: dict(n=v["n"], ms=round(v["ms"], 4)) for k, v in agg.items()})
    if not args.no_cpu_baseline:
        cb, lz_o, marg_o = cpu_baseline(net)
        out["cpu_baseline"] = cb
        got = plan.split_marginals(m[0])
        out["err_vs_oracle"] = dict(
            log_z_rel=abs(float(lz[0]) - lz_o) / abs(lz_o),
            marginal_max_abs=float(max(np.abs(a - b).max() for a, b in zip(got, marg_o))))
        out["speedup_vs_cpu_oracle"] = round(solves_per_s / cb["value"], 1)
    if args.copy_probe:
        # 256 MiB source, then 2 GiB of other writes so the source is not
        # cache resident, then copies: each reads and writes 256 MiB
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        flush = torch.empty(512 << 20, dtype=torch.float32, device="cuda")
        flush.fill_(2.0)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
            flush.fill_(3.0)
        torch.cuda.synchronize()
        del flush
        out["copy_probe_bytes"] = 2 * x.numel() * 4
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
