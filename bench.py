#!/usr/bin/env python
"""Benchmark of the hot path (one GPU).

Default workload (the metric's configuration): the 20x20 binary grid MRF
(400 variables, 400 unary + 760 pairwise Gaussian log-potential tables,
seed 0), contracted along the library's planned tree (bucket elimination,
largest intermediate 2^20 elements).  One step = one call of tn_marginals:
leaf preparation, the forward sum-product over the tree, the reverse pass and
the marginal normalisation, results copied back to the host.  Factor tables
are resident in device memory before the timed region.

Other workloads (--workload), each printed as the same kind of JSON line:
  bn500x512   500-variable Bayesian network, 512 evidence sets in one batched
              indicator pass (log Z + all marginals of every instance); the
              plain FP32 per-instance form is timed beside it
  bn300_map   300-variable Bayesian network, 30 observed: MAP (max-plus
              contraction + argmax readout), checked bit for bit against the
              oracle's FP32 emulation
  grid20_map  MAP on the 20x20 grid (max-plus at the size of the sum-product
              workload)
  regular3_mmap  MMAP on the 220-variable 3-regular graph (25 query variables,
              sliced to intermediates <= 2^28) and 10k samples
  tropical_gemm  MAP on a three-factor network whose time is one dense
              max-plus product (4 x 729^3 candidates, argmax kept), against
              the vector-ALU bound

Prints one JSON line.
"""
import argparse
import hashlib
import json
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
              7: "seg_carrier_bwd", 8: "seg_maps", 9: "seg_adjoint_sweeps", 10: "contract_mfma_sum",
              11: "contract_tropical_dense", 12: "contract_interleaved_sum", 13: "contract_interleaved_max"}

# HBM bytes per launch of a kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counter runs (scaled by the counts of a plain 256 MiB copy), valid only for
# the kernel source they were taken from (sha256 prefix of tn_kernels.hip):
# {(kernel, workload): {"src": sha, "bytes": B}}
MEASURED_TRAFFIC = {
    ("seg_carrier_bwd", "grid20x20"): {"src": "057dbbc795256e42", "bytes": 26376110},
    ("contract_interleaved_sum", "bn500x512"): {"src": "057dbbc795256e42", "bytes": 70048750},
    ("contract_map_max", "grid20_map"): {"src": "057dbbc795256e42", "bytes": 20524736},
    ("contract_tropical_dense", "tropical_gemm"): {"src": "057dbbc795256e42", "bytes": 115420100},
}

def kernel_src_sha():
    with open(os.path.join(ROOT, "paper_2405_14060_amd", "csrc", "tn_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_summary(prof):
    agg = {}
    for kind, fl, by, ms in prof:
        a = agg.setdefault(KIND_NAMES[kind], dict(n=0, flops=0.0, bytes=0.0, ms=0.0))
        a["n"] += 1
        a["flops"] += fl
        a["bytes"] += by
        a["ms"] += ms
    return agg


def roofline(plan, task, workload, evidence=None, batch=1, kernel=None):
    """Dominant kernel kind of one task by executed time (or the named kind);
    its launches timed back to back between two HIP events on the plan's
    stream."""
    prof = plan.profile(task, reps=3, evidence=evidence, batch=batch)
    agg = kernel_summary(prof)
    flops_task = sum(fl for _, fl, _, _ in prof)
    dom_name = kernel or max(agg.items(), key=lambda kv: kv[1]["ms"])[0]
    kind_of = {v: k for k, v in KIND_NAMES.items()}
    avg_ms, fl_launch, by_launch, n_launch = plan.profile_kind(task, kind_of[dom_name], reps=5,
                                                               evidence=evidence, batch=batch)
    achieved_gbs = by_launch / (avg_ms * 1e-3) / 1e9
    achieved_tf = fl_launch / (avg_ms * 1e-3) / 1e12
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    mfma_frac = achieved_tf / FP32_PEAK_TFLOPS
    meas = MEASURED_TRAFFIC.get((dom_name, workload))
    traffic = meas["bytes"] if meas and meas["src"] == kernel_src_sha() else None
    if hbm_frac >= mfma_frac:
        roof = dict(bound="hbm", achieved=round(achieved_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(hbm_frac, 4), traffic=traffic)
    else:
        roof = dict(bound="mfma", achieved=round(achieved_tf, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(mfma_frac, 4), traffic=traffic)
    roof.update(kernel=dom_name, launches_per_solve=n_launch, avg_launch_us=round(avg_ms * 1e3, 3),
                bytes_per_launch=round(by_launch), flops_per_launch=round(fl_launch))
    if roof["bound"] == "hbm":
        roof["copy_ref"] = copy_reference(by_launch)
    kernels = {k: dict(n=v["n"], ms=round(v["ms"], 4)) for k, v in agg.items()}
    return roof, kernels, flops_task


def copy_reference(nbytes, reps=50):
    """What one launch moving the same bytes reaches: a plain device copy of
    nbytes / 2 bytes (read once, written once), launched back to back like the
    kernel kinds (one graph of `reps` copies, replayed between two events on
    the same stream).  "hbm":
    each launch copies another pair of slices of a 1 GiB pool (source and
    destination out of the caches); "cached": one pair of buffers every time
    (both stay in the last-level cache, as a pass's freshly written carriers
    may)."""
    import torch
    n = max(1, int(nbytes // 8))
    slots = max(2, (1 << 28) // n)  # 1 GiB of floats per pool
    src = torch.ones(slots * n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, rot in (("hbm", True), ("cached", False)):
        views = [((r % slots) * n if rot else 0) for r in range(reps)]
        pairs = [(dst[k:k + n], src[k:k + n]) for k in views]
        for d, c in pairs[:5]:
            d.copy_(c)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()  # the copies replay back to back, free of host overhead
        with torch.cuda.graph(g):
            for d, c in pairs:
                d.copy_(c)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        del g
        out[name] = dict(us=round(us, 3), frac=round(8 * n / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
    del src, dst
    out["what"] = "plain device copy of the launch's byte count (half read, half written), one launch each"
    return out


def timed(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    sync()
    return (time.perf_counter() - t0) / steps, out


def step_stats(fn, np, reps=50):
    """Wall times of `reps` further calls, each timed alone: the calls return
    their results in host memory, so one call is one whole solve end to end
    (launch, kernels, copies back).  Median and 10th / 90th percentiles in ms."""
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    p10, med, p90 = np.percentile(np.array(ts) * 1e3, [10, 50, 90])
    return dict(reps=reps, p10=round(float(p10), 4), median=round(float(med), 4), p90=round(float(p90), 4))


def bench_grid20(args, T, W, np, sync):
    net = W.grid_mrf(20, 20, 0)
    dt = dict(f32=T.TN_F32, bf16=T.TN_BF16, f16=T.TN_F16)[args.dtype]
    plan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, use_graph=not args.no_graph, dtype=dt,
                  autotune=args.autotune)
    info = plan.info()
    sec, (lz, m) = timed(plan.marginals, args.steps, args.warmup, lambda: (plan.sync(), sync()))
    roof, kernels, flops = roofline(plan, 1, "grid20x20")
    out = dict(value=round(1.0 / sec, 3), unit="solves/s", ms_per_step=round(sec * 1e3, 4),
               dtype=args.dtype,
               config=dict(workload="grid20x20_mrf logZ+all-marginals", seed=0, n_vars=400, n_factors=1160,
                           tree_sc_log2=info["sc"], tree_tc_log2=round(info["tc"], 3),
                           segments=info["n_segments"], launches_per_solve=info["n_launches_fwd"] +
                           info["n_launches_bwd"] + 3, graph=not args.no_graph, autotune=args.autotune),
               tflops=round(flops / sec / 1e12, 4), log_z=float(lz[0]), roofline=roof, kernels=kernels,
               step_ms=step_stats(plan.marginals, np))
    if not args.no_cpu_baseline:
        import oracle
        lv = oracle.build_leaves(net)
        pairs = oracle.elimination_tree(lv.labels, lv.card, list(range(net.n_vars)))
        t0 = time.perf_counter()
        lz_o, marg_o, *_ = oracle.marginals(net, pairs=pairs)
        d = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=1.0 / d, unit="solves/s", cores=oracle.threads(), kind="oracle",
                                   sample="one full solve (log Z + all 400 marginals) of the same 20x20 grid, "
                                          "FP64 loop nests, output elements of each contraction split over "
                                          "%d threads (OpenMP), %.1f s" % (oracle.threads(), d))
        got = plan.split_marginals(m[0])
        out["err_vs_oracle"] = dict(log_z_rel=abs(float(lz[0]) - lz_o) / abs(lz_o),
                                    marginal_max_abs=float(max(np.abs(a - b).max() for a, b in zip(got, marg_o))))
        out["speedup_vs_cpu_oracle"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    return out


def bench_bn500x512(args, T, W, np, sync):
    c = W.config(3, 0)
    net, ev = c["net"], c["evidence"]
    B = ev.shape[0]
    dt = dict(f32=T.TN_F32, bf16=T.TN_BF16, f16=T.TN_F16)[args.dtype]
    layout = dict(auto=T.LAYOUT_AUTO, instance_major=T.LAYOUT_INSTANCE_MAJOR,
                  interleaved=T.LAYOUT_INTERLEAVED)[args.batch_layout]
    plan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=B,
                  use_graph=not args.no_graph, dtype=dt, autotune=args.autotune, batch_layout=layout)
    info = plan.info()
    sec, (lz, m) = timed(lambda: plan.marginals(ev, batch=B), args.steps, args.warmup,
                         lambda: (plan.sync(), sync()))
    roof, kernels, flops = roofline(plan, 1, "bn500x512", evidence=ev, batch=B)
    steps = step_stats(lambda: plan.marginals(ev, batch=B), np)
    # the plain FP32 per-instance form: one instance per call, no batching
    one = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=1,
                 use_graph=not args.no_graph)
    n1 = 32
    sec1, _ = timed(lambda: [one.marginals(ev[b:b + 1], batch=1) for b in range(n1)], 1, 1,
                    lambda: (one.sync(), sync()))
    lz1 = np.array([one.marginals(ev[b:b + 1], batch=1)[0][0] for b in range(4)])
    # the batched form with BF16 operands on the matrix cores (instance-major
    # layout, dense contractions on MFMA, FP32 accumulation and storage)
    lp_plan = None
    if args.dtype == "f32":
        lp_plan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, evidence_mode=T.EVIDENCE_INDICATOR, max_batch=B,
                         use_graph=not args.no_graph, dtype=T.TN_BF16, batch_layout=T.LAYOUT_INSTANCE_MAJOR)
        sec_lp, (lz_lp, m_lp) = timed(lambda: lp_plan.marginals(ev, batch=B), max(3, args.steps // 2), args.warmup,
                                      lambda: (lp_plan.sync(), sync()))
    out = dict(value=round(B / sec, 1), unit="instance-solves/s", ms_per_step=round(sec * 1e3, 4),
               dtype=args.dtype,
               config=dict(workload="bn500 x 512 evidence sets, logZ+all-marginals, batched indicator pass",
                           seed=0, n_vars=500, batch=B, tree_sc_log2=round(info["sc"], 3),
                           tree_tc_log2=round(info["tc"], 3), dense_nodes=info["n_dense"],
                           wave_nodes=info["n_wave"], interleaved_nodes=info["n_interleaved"],
                           batch_layout="interleaved" if info["batch_stride"] else "instance_major",
                           graph=not args.no_graph, autotune=args.autotune),
               tflops=round(flops / sec / 1e12, 4), roofline=roof, kernels=kernels, step_ms=steps,
               per_instance_fp32=dict(value=round(n1 / sec1, 2), unit="instance-solves/s",
                                      max_log_z_diff_vs_batched=float(np.abs(lz1 - lz[:4]).max())))
    if lp_plan is not None:
        out["batched_bf16_mfma"] = dict(value=round(B / sec_lp, 1), unit="instance-solves/s",
                                        ms_per_step=round(sec_lp * 1e3, 4), layout="instance_major",
                                        dense_nodes=lp_plan.info()["n_dense"])
    if not args.no_cpu_baseline:
        import oracle
        n_o, t0 = 0, time.perf_counter()
        errs, errs_lp = [], []
        while n_o < 64 and time.perf_counter() - t0 < 20.0:
            lz_o, marg_o, *_ = oracle.marginals(net, ev[n_o], mode="indicator")
            got = plan.split_marginals(m[n_o])
            errs.append((abs(lz[n_o] - lz_o) / max(1.0, abs(lz_o)),
                         max(np.abs(a - b).max() for a, b in zip(got, marg_o))))
            if lp_plan is not None:
                got = lp_plan.split_marginals(m_lp[n_o])
                errs_lp.append((abs(lz_lp[n_o] - lz_o) / max(1.0, abs(lz_o)),
                                max(np.abs(a - b).max() for a, b in zip(got, marg_o))))
            n_o += 1
        d = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=n_o / d, unit="instance-solves/s", cores=oracle.threads(), kind="oracle",
                                   sample="first %d of the 512 evidence sets, FP64 loop nests over %d threads "
                                          "(OpenMP), %.1f s" % (n_o, oracle.threads(), d))
        out["err_vs_oracle"] = dict(log_z_rel=float(max(e[0] for e in errs)),
                                    marginal_max_abs=float(max(e[1] for e in errs)), instances=n_o)
        if errs_lp:
            out["batched_bf16_mfma"]["err_vs_oracle"] = dict(
                log_z_rel=float(max(e[0] for e in errs_lp)), marginal_max_abs=float(max(e[1] for e in errs_lp)),
                instances=n_o)
    return out


def bench_regular3_mmap(args, T, W, np, sync):
    """MMAP on the 220-variable 3-regular graph (25 query variables), tree
    sliced so that no intermediate exceeds 2^28 entries: the whole query
    (every slice of the sum phase, then the max phase and the readout) timed
    end to end; one slice profiled launch by launch for the roofline."""
    c = W.config(4, 0)
    net, q = c["net"], c["query"]
    tp = time.perf_counter()
    plan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT | T.MAX_PLUS, query=q, max_log2_size=28,
                  use_graph=False, autotune=args.autotune, restarts=args.restarts)
    plan_s = time.perf_counter() - tp
    info = plan.info()
    print("regular3_mmap: planned in %.1f s (2^%.2f multiply-adds, %d slices)" % (plan_s, info["tc"], 2 ** info["n_sliced"]),
          file=sys.stderr, flush=True)
    n_slices = 2 ** info["n_sliced"]
    if not args.slice_only:
        t0 = time.perf_counter()
        val, x = plan.mmap()
        sync()
        sec = time.perf_counter() - t0
    prof = plan.profile(3, reps=1)
    slice_s = sum(ms for _, _, _, ms in prof) / 1e3
    # measured HBM traffic belongs to one plan: the tree search's restarts are part of the key (with
    # 1024 restarts the autotuner's form choices, and so the slice's launches, differ between processes:
    # no figure is kept for that plan)
    wl = "regular3_220_r%d" % args.restarts
    roof, kernels, slice_flops = roofline(plan, 3, wl)
    # the matrix-core kernel of the slice against the FP32 matrix-core peak
    roof_dense = roofline(plan, 3, wl, kernel="contract_mfma_sum")[0]
    if args.slice_only:  # profiling aid: one slice, time of the query projected from it
        return dict(value=1.0 / (slice_s * n_slices), unit="MMAP solves/s (projected from one slice)",
                    ms_per_step=round(slice_s * n_slices * 1e3, 1), dtype="f32",
                    config=dict(workload="regular3 220 vars, MMAP with 25 query vars, intermediates <= 2^28 "
                                "(sliced), one slice", seed=0, n_slices=n_slices, autotune=args.autotune,
                                restarts=args.restarts),
                    slice_ms=round(slice_s * 1e3, 3), roofline=roof, roofline_dense=roof_dense,
                    kernels_one_slice=kernels)
    # certificate at full size: log p(Q = x) by the oracle (the network with
    # the query variables observed is small) equals the reported value
    import oracle
    ev = -np.ones(net.n_vars, np.int32)
    ev[np.asarray(q)] = x
    t1 = time.perf_counter()
    lp_oracle = oracle.log_z(net, ev, mode="slice")
    t_oracle_cert = time.perf_counter() - t1
    out = dict(value=1.0 / sec, unit="MMAP solves/s", ms_per_step=round(sec * 1e3, 1), dtype="f32",
               config=dict(workload="regular3 220 vars, MMAP with 25 query vars, intermediates <= 2^28 (sliced)",
                           seed=0, n_vars=220, n_query=len(q), n_sliced=info["n_sliced"], n_slices=n_slices,
                           tree_sc_log2=round(info["sc"], 3), tree_tc_log2=round(info["tc"], 3),
                           device_gb=round(info["device_bytes"] / 1e9, 2), graph=False, autotune=args.autotune,
                           restarts=args.restarts, plan_s=round(plan_s, 1)),
               log_value=val, slice_ms=round(slice_s * 1e3, 3), tflops=round(slice_flops / slice_s / 1e12, 3),
               roofline=roof, roofline_dense=roof_dense, kernels_one_slice=kernels,
               certificate=dict(oracle_log_p_of_answer=lp_oracle, abs_diff=abs(lp_oracle - val),
                                oracle_s=round(t_oracle_cert, 1)))
    # the same network without the query: log Z and 10k samples from a
    # sum-product plan sliced to the same cap (each sample draws its slice
    # with probability Z_s / Z, then the per-node rule inside it)
    tp = time.perf_counter()
    splan = T.Plan(T.Network(net), semirings=T.SUM_PRODUCT, max_log2_size=28, restarts=args.sample_restarts,
                   autotune=args.autotune)
    splan_s = time.perf_counter() - tp
    sinfo = splan.info()
    print("regular3_mmap: sampling plan in %.1f s (2^%.2f multiply-adds)" % (splan_s, sinfo["tc"]), file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    lz = splan.log_z()[0]
    t_lz = time.perf_counter() - t0
    t0 = time.perf_counter()
    smp = splan.sample(10000, seed=1)
    t_s = time.perf_counter() - t0
    out["sampling"] = dict(n=10000, seconds=round(t_s, 2), samples_per_s=round(10000 / t_s, 1), log_z=lz,
                           log_z_seconds=round(t_lz, 2), n_sliced=sinfo["n_sliced"],
                           tree_tc_log2=round(sinfo["tc"], 3), restarts=args.sample_restarts,
                           plan_s=round(splan_s, 1),
                           complete=bool(np.all(smp >= 0)))
    if not args.no_cpu_baseline:
        qs = set(int(v) for v in q)
        summed = [v for v in range(net.n_vars) if v not in qs]
        k = 44
        fix = list(np.random.default_rng(1).permutation(summed)[:k])
        ev = -np.ones(net.n_vars, np.int32)
        ev[fix] = 0
        lv = oracle.build_leaves(net, ev, "slice")
        order = [v for v in oracle.min_degree_order(lv.labels, net.n_vars) if v not in qs]
        pairs = oracle.elimination_tree(lv.labels, lv.card, order)
        st = oracle.tree_stats(lv.labels, pairs, lv.card, out=np.sort(q))
        t0 = time.perf_counter()
        oracle.sum_forward(lv, pairs, out=np.sort(q))
        d = time.perf_counter() - t0
        mac_rate = 2.0 ** st["tc"] / d
        out["cpu_baseline"] = dict(value=mac_rate / 2.0 ** info["tc"], unit="MMAP solves/s (projected)",
                                   cores=oracle.threads(),
                                   kind="oracle",
                                   sample="oracle sum phase of one sub-slice (%d summed variables fixed, its own "
                                          "tree, 2^%.2f multiply-adds, %.1f s, FP64 over all host threads); projected to "
                                          "the plan's 2^%.2f multiply-adds at the same rate" % (k, st["tc"], d,
                                                                                               info["tc"]))
    return out


# dense max-plus on the vector ALUs: one candidate is one FP32 add and one
# max (2 tropical ops, as a sum-product candidate is a multiply and an add);
# each is one non-packed VALU instruction per lane, and the chip issues
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T such lane-operations per
# second.  Keeping the argmax costs a compare and a second select per
# candidate on top of that (the fraction is against the value-only bound).
TROPICAL_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def bench_tropical_gemm(args, T, W, np, sync):
    """MAP on a three-factor network whose max-plus tree starts with one
    large dense tropical product Z[b, m, n] = max_s X[b, m, s] + Y[b, s, n]
    (4 x 729 x 729 x 729 candidates), with its argmax; then the small
    remainder of the tree and the argmax readout."""
    net = W.three_factor_net(2, 6, 6, 6, 3, seed=0)
    plan = T.Plan(T.Network(net), semirings=T.MAX_PLUS, use_graph=not args.no_graph)
    info = plan.info()
    sec, (lp, x) = timed(lambda: plan.map(), args.steps, args.warmup, lambda: (plan.sync(), sync()))
    steps = step_stats(plan.map, np)
    prof = plan.profile(2, reps=3)
    kind_of = {v: k for k, v in KIND_NAMES.items()}
    avg_ms, fl_launch, by_launch, n_launch = plan.profile_kind(2, kind_of["contract_tropical_dense"], reps=5)
    tops = fl_launch / (avg_ms * 1e-3) / 1e12
    meas = MEASURED_TRAFFIC.get(("contract_tropical_dense", "tropical_gemm"))
    traffic = meas["bytes"] if meas and meas["src"] == kernel_src_sha() else None
    roof = dict(bound="alu", achieved=round(tops, 3), peak=round(TROPICAL_PEAK_TOPS, 2), unit="T tropical-op/s",
                frac=round(tops / TROPICAL_PEAK_TOPS, 4), traffic=traffic, kernel="contract_tropical_dense",
                launches_per_solve=n_launch, avg_launch_us=round(avg_ms * 1e3, 3), bytes_per_launch=round(by_launch),
                flops_per_launch=round(fl_launch), candidates_per_s=round(fl_launch / 2 / (avg_ms * 1e-3), 1))
    kernels = {k: dict(n=v["n"], ms=round(v["ms"], 4)) for k, v in kernel_summary(prof).items()}
    out = dict(value=round(1.0 / sec, 3), unit="MAP solves/s", ms_per_step=round(sec * 1e3, 4), dtype="f32",
               config=dict(workload="three-factor network, 4 x 729 x 729 x 729 dense max-plus product + readout",
                           seed=0, n_vars=int(net.n_vars), tree_sc_log2=round(info["sc"], 3),
                           tree_tc_log2=round(info["tc"], 3), graph=not args.no_graph),
               log_p=float(lp[0]), roofline=roof, kernels=kernels, step_ms=steps)
    if not args.no_cpu_baseline:
        import oracle
        pairs, _ = plan.tree()
        t0 = time.perf_counter()
        val, asg = oracle.map_assignment(net, None, pairs=pairs.astype(np.int64), fp32=True)
        d = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=1.0 / d, unit="MAP solves/s", cores=1, kind="oracle",
                                   sample="one MAP solve on the plan's tree, FP32-emulating loops, %.1f s" % d)
        out["bit_exact_vs_oracle_fp32"] = bool(np.array_equal(np.asarray(asg), x[0]) and
                                               np.float32(val) == np.float32(lp[0]))
    return out


def bench_map(args, T, W, np, sync, which):
    if which == "bn300_map":
        c = W.config(2, 0)
        net, obs, ev = c["net"], c["observed"], c["evidence"]
        plan = T.Plan(T.Network(net), semirings=T.MAX_PLUS, evidence_mode=T.EVIDENCE_SLICED, observed=obs,
                      use_graph=not args.no_graph)
        evb = ev.reshape(1, -1)
        wl = "bn300 MAP, 30 observed (max-plus + argmax readout)"
    else:
        net, ev, evb = W.grid_mrf(20, 20, 0), None, None
        plan = T.Plan(T.Network(net), semirings=T.MAX_PLUS, use_graph=not args.no_graph)
        wl = "grid20x20 MAP (max-plus + argmax readout)"
    info = plan.info()
    sec, (lp, x) = timed(lambda: plan.map(evb), args.steps, args.warmup, lambda: (plan.sync(), sync()))
    roof, kernels, flops = roofline(plan, 2, which, evidence=evb)
    out = dict(value=round(1.0 / sec, 3), unit="MAP solves/s", ms_per_step=round(sec * 1e3, 4), dtype="f32",
               config=dict(workload=wl, seed=0, n_vars=int(net.n_vars), tree_sc_log2=round(info["sc"], 3),
                           tree_tc_log2=round(info["tc"], 3), graph=not args.no_graph),
               tflops=round(flops / sec / 1e12, 4), log_p=float(lp[0]), roofline=roof, kernels=kernels,
               step_ms=step_stats(lambda: plan.map(evb), np))
    if not args.no_cpu_baseline:
        import oracle
        pairs, _ = plan.tree()
        t0 = time.perf_counter()
        val, asg = oracle.map_assignment(net, ev, pairs=pairs.astype(np.int64), fp32=True)
        d = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=1.0 / d, unit="MAP solves/s", cores=1, kind="oracle",
                                   sample="one MAP solve on the plan's tree, FP32-emulating loops, %.1f s" % d)
        out["bit_exact_vs_oracle_fp32"] = bool(np.array_equal(np.asarray(asg), x[0]) and np.float32(val) == np.float32(lp[0]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid20", choices=["grid20", "bn500x512", "bn300_map", "grid20_map",
                                                               "regular3_mmap", "tropical_gemm"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"],
                    help="matrix-core operand precision of the sum-product workloads")
    ap.add_argument("--batch-layout", default="auto", choices=["auto", "instance_major", "interleaved"],
                    help="batched workload: layout of the instances (auto: interleaved for f32)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="pick kernel forms by the fixed rules instead of timing the eligible forms of every "
                         "contraction shape at plan time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--restarts", type=int, default=1024,
                    help="regular3_mmap: randomised restarts of the MMAP plan's tree search (plan time only; "
                         "the query's sliced work: 2^47.1 multiply-adds at 16, 2^43.4 at 1024)")
    ap.add_argument("--sample-restarts", type=int, default=256,
                    help="regular3_mmap: restarts of the sampling (log Z) plan's tree search (2^39.8 "
                         "multiply-adds in 512 slices at 16, 2^41.1 in 8 slices at 256)")
    ap.add_argument("--slice-only", action="store_true",
                    help="regular3_mmap: plan and profile one slice only (for profilers)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; a run on several GPUs would shard the work by evidence "
              "instance or by slice, and is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2405_14060_amd as T
    from paper_2405_14060_amd import workloads as W

    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    if args.workload == "grid20":
        res = bench_grid20(args, T, W, np, sync)
    elif args.workload == "bn500x512":
        res = bench_bn500x512(args, T, W, np, sync)
    elif args.workload == "regular3_mmap":
        res = bench_regular3_mmap(args, T, W, np, sync)
    elif args.workload == "tropical_gemm":
        res = bench_tropical_gemm(args, T, W, np, sync)
    else:
        res = bench_map(args, T, W, np, sync, args.workload)
    out = dict(metric=METRIC, value=res.pop("value"), unit=res.pop("unit"), n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=res.pop("ms_per_step"), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=res.pop("dtype"), data="synthetic", config=res.pop("config"))
    out.update(res)
    if args.copy_probe:
        # 256 MiB source, then 2 GiB of other writes so the source is not
        # cache resident, then copies: each reads and writes 256 MiB
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        flush = torch.empty(512 << 20, dtype=torch.float32, device="cuda")
        flush.fill_(2.0)
        sync()
        for _ in range(3):
            y.copy_(x)
            flush.fill_(3.0)
        sync()
        del flush
        out["copy_probe_bytes"] = 2 * x.numel() * 4
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
