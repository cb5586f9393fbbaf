#!/usr/bin/env python3
"""Benchmark of the treecode evaluation phase on one MI355X.

Workload (the headline configuration): N = 1,000,000 particles uniform in
[-1, 1]^3, targets = sources, charges uniform in [-1, 1], Coulomb kernel,
theta = 0.7, degree n = 8, N_L = N_B = 2000, seeded synthetic inputs.

A step is one evaluation with the geometry fixed (plan built once, outside the
timed region): charges gathered into tree order, upward pass (eqs. 14-15), all
batch/cluster interactions (eqs. 9, 11), potentials written in caller order.
Inputs are resident in HBM when the timed region starts.

Prints one JSON line (rank 0).  Errors are measured on sampled targets against
the FP64 CPU oracle (treecode and direct sum), which is also timed on the
host's cores as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X: 256 CU x 64 lanes x 2 flops x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak (packed FP32)
# Flop convention per kernel value (one target, one source or proxy point):
# Coulomb 9 flops + 1 reciprocal square root = 10; Yukawa adds 1 exponential and
# 2 flops = 13.  A mutual direct pair (targets = sources) forms one kernel value
# that serves the row and the column term: + 1 multiply-add (2).
FLOPS_COULOMB = 10
FLOPS_YUKAWA = 13
FLOPS_PAIR_EXTRA = 2
# Hermite approximation, per grid point and target (Coulomb): distance 8, reciprocal
# square root 1, g1..g3 from 1/r 6, d1 d2 and d1 d2 d3 2, first-order sum 5,
# second-order sum 6, third-order product 1, combination with g0..g3 7, accumulate 1
FLOPS_HERMITE_POINT = 37
FLOPS_MUTUAL_PAIR = FLOPS_COULOMB + FLOPS_PAIR_EXTRA

MFMA_F64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 matrix peak
KERNEL_SOURCES = {
    "upward_single": ["kernels_upward.hip", "kernels.hpp"],
    "interact_mixed": ["kernels_mixed.hip", "device_mixed.hpp", "device_common.hpp", "kernels.hpp"],
    "interact_f64": ["kernels.hip", "device_common.hpp", "kernels.hpp"],
    "near_pairs_mixed": ["kernels_sym.hip", "device_common.hpp", "kernels.hpp"],
    "near_pairs_f64": ["kernels_sym.hip", "device_common.hpp", "kernels.hpp"],
}


# Issue-rate model of the interaction kernels: core cycles per wave instruction
# (64 lanes) from paper_2003_01836_amd/microbench (8 independent chains per
# lane, 16 waves per SIMD; its wall time times the clock that GRBM_GUI_ACTIVE
# reports for the same dispatch, profiles/issue_rates_microbench.md): FP32
# FMA-class and other 32-bit instructions, the FP32 transcendentals (v_rsq_f32,
# v_exp_f32), FP64 add / multiply / FMA, and v_rsq_f64.  Their issue adds up.
CYCLES_FMA32 = 2.54
CYCLES_TRANS32 = 8.8
CYCLES_F64 = 4.4
CYCLES_TRANS64 = 16.6
SIMDS = 1024                        # 256 CU x 4 SIMD
CLOCK_HZ = 2.4e9                    # nominal; the model takes the kernel's measured clock


def counter_value(prefix, profile, kernel, degree, ker_id, tpt=1):
    """A per-launch value of `kernel` from a committed rocprofv3 summary (lines
    `<prefix> <kernel instantiation> <value> source <hash> [tpt <threads per target>]`,
    measured with that many threads per target, 1 when absent), or None when there
    is none for this instantiation and threads per target or the kernel's sources
    changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2003_01836_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if kernel == "upward_single":
        # ker_id 1: the FP32-product instantiation of the FP32-mixed path
        want = f"{prefix} {kernel}<{degree + 1}, false, {'true' if ker_id else 'false'}> "
    elif kernel.startswith("interact"):
        want = f"{prefix} {kernel}<{degree}, {ker_id}> "
    else:
        want = f"{prefix} {kernel}<{ker_id}> "
    with open(path) as fh:
        for line in fh:
            if line.startswith(want):
                parts = line[len(want):].split()
                if len(parts) == 5 and parts[3] == "tpt":
                    line_tpt = int(parts[4])
                    parts = parts[:3]
                else:
                    line_tpt = 1
                if (len(parts) == 3 and parts[1] == "source" and parts[2] == h.hexdigest()[:16]
                        and line_tpt == tpt):
                    return float(parts[0])
    return None


def counter_traffic(kernel, degree, ker_id, tpt=1):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, calibrated by a plain copy)."""
    return counter_value("traffic_bytes", "interact_uniform-1M_counters.md", kernel, degree,
                         ker_id, tpt)


def issue_model(kernel, degree, ker_id, trans_per_eval, evals, ms, tpt=1):
    """Shortest time at which the SIMDs could issue the VALU instructions that the
    kernel issues per launch, from the committed counter summary (SQ_INSTS_VALU; for
    the FP32-mixed kernels the FP32 transcendentals, one per kernel value or two for
    Yukawa where no counter run took them; for the FP64 kernels the FP64 add, multiply
    and FMA instructions and v_rsq_f64), each class at its probed issue cost, the rest
    at the 32-bit rate, at the kernel's clock from the same summary (GRBM_GUI_ACTIVE
    over its time; nominal 2.4 GHz where none was taken); and its ratio to the
    measured launch time.  None where no counters fit the kernel."""
    prof = "interact_uniform-1M_valu_counters.md"
    valu = counter_value("valu_insts", prof, kernel, degree, ker_id, tpt)
    if valu is None:
        return None
    if kernel.endswith("mixed"):
        trans = counter_value("trans_insts", prof, kernel, degree, ker_id, tpt)
        if trans is None:
            trans = trans_per_eval * evals / 64.0
        cycles = (valu - trans) * CYCLES_FMA32 + trans * CYCLES_TRANS32
        parts = {"trans_insts": trans}
    else:
        f64 = counter_value("f64_insts", prof, kernel, degree, ker_id, tpt)
        trans = counter_value("trans64_insts", prof, kernel, degree, ker_id, tpt)
        if f64 is None or trans is None:
            return None
        cycles = f64 * CYCLES_F64 + trans * CYCLES_TRANS64 + (valu - f64 - trans) * CYCLES_FMA32
        parts = {"f64_insts": f64, "trans64_insts": trans}
    clock = counter_value("clock_hz", prof, kernel, degree, ker_id, tpt) or CLOCK_HZ
    t_min = cycles / SIMDS / clock * 1e3
    return {"valu_insts": valu, **parts, "clock_hz": clock, "t_min_ms": t_min, "frac": t_min / ms}


def upward_roofline(degree, macs, ms, prec="fp64"):
    """The upward pass of one charge vector against the matrix-core peak of its
    products (FP64 for the FP64 path, FP32 for the FP32-mixed one): algorithmic flops
    2 * sum_C N_C (n+1)^3 over the phase time (the kernel and the chunk-sum
    reduction), and the matrix-core busy time per SIMD from the committed counter
    summary (None when the kernel changed since)."""
    f32 = prec != "fp64"
    peak = FP32_VECTOR_PEAK_TFLOPS if f32 else MFMA_F64_PEAK_TFLOPS
    achieved = 2.0 * macs / (ms * 1e-3) / 1e12
    busy = counter_value("mfma_busy_cycles", "upward_uniform-1M_mfma_counters.md",
                         "upward_single", degree, 1 if f32 else 0)
    return {"kernel": f"upward_single<{degree + 1}, false, {'true' if f32 else 'false'}>",
            "bound": "mfma", "macs": macs, "ms": ms, "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "mfma_busy_frac": None if busy is None else busy / SIMDS / (ms * 1e-3 * CLOCK_HZ)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rel_l2(ref, got):
    import numpy as np
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    return float(np.sqrt(np.sum((ref - got) ** 2) / np.sum(ref * ref)))


WORKLOADS = {
    "uniform-1M": dict(n=1_000_000, dist="uniform", theta=0.7, degree=8, leaf=2000, batch=2000,
                       kernel="coulomb", kappa=0.0, cfg=1, samples=1000),
    "uniform-10K": dict(n=10_000, dist="uniform", theta=0.7, degree=4, leaf=500, batch=500,
                        kernel="coulomb", kappa=0.0, cfg=0, samples=1000),
}


def run_batched(args, dev):
    """64 independent systems (sizes log-uniform in [1e4, 1e6], uniform cubes), 16 charge
    vectors each, theta 0.7, n 8, leaf/batch size from the library's autotuner, one
    persistent work-queue launch per evaluation replayed from a hipGraph."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    prec = "fp32_mixed" if args.precision == "fp32_mixed" else "fp64"
    sizes = inputs.log_uniform_sizes(64, inputs.config_seed(3))
    log(f"batched: {len(sizes)} systems, {int(sizes.sum())} particles, 16 vectors, {prec}")
    plans, qs, outs, pos_all, q_all, leaves = [], [], [], [], [], []
    t_tune = 0.0
    for k, n in enumerate(sizes):
        pos, q = inputs.uniform_cube(int(n), inputs.config_seed(3) * 100 + k, m=16)
        t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
        t0 = time.perf_counter()
        leaf, _ = bltc.autotune(t, t, (1000, 2000, 3000, 4000), num_q=16, theta=0.7, degree=8,
                                precision=prec)
        t_tune += time.perf_counter() - t0
        leaves.append(leaf)
        plans.append(bltc.Plan(t, t, theta=0.7, degree=8, leaf_size=leaf, batch_size=leaf,
                               precision=prec, max_q=16))
        qs.append(torch.from_numpy(q).to(dev))
        outs.append(torch.empty((16, int(n)), dtype=torch.float64, device=dev))
        pos_all.append(pos)
        q_all.append(q)
    batch = bltc.Batch(plans)
    for _ in range(args.warmup):
        batch.execute(qs, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.execute(qs, outs)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    total = int(sizes.sum())
    errs = []
    if not args.no_cpu:
        import oracle
        # every fourth system, 4 of its 16 vectors, 200 sampled targets each
        vec = [0, 5, 10, 15]
        for k in range(0, 64, 4):
            smp = inputs.sample_indices(int(sizes[k]), 200, inputs.sample_seed(3) + k)
            oc = oracle.Treecode(pos_all[k], pos_all[k], 0.7, 8, leaves[k], leaves[k])
            ref = oc.potential(q_all[k][vec], sample=smp)
            got = outs[k][vec].cpu().numpy()[:, smp]
            errs.append(max(rel_l2(ref[i], got[i]) for i in range(len(vec))))
            log(f"batched: system {k} ({int(sizes[k])} particles) E_par {errs[-1]:.2e}")
    info = batch.info()
    # a kernel value G(x, y) (VALU, 11 flops) serves the 16 vectors through the
    # matrix cores (16 multiply-adds); priced over the whole step
    far_values = sum(p.stats()["far_evals"] for p in plans)
    near_values = sum(p.stats()["near_evals"] for p in plans)
    values = far_values + near_values
    t_s = ms * 1e-3
    peak = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    mpeak = MFMA_F64_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    roof = {"bound": "alu", "achieved": values * FLOPS_COULOMB / t_s / 1e12, "peak": peak,
            "unit": "TFLOP/s", "frac": values * FLOPS_COULOMB / t_s / 1e12 / peak,
            "traffic": None, "kernel": "interact_queue (whole step)", "kernel_values": values,
            "contraction": {"bound": "mfma", "achieved": values * 32 / t_s / 1e12,
                            "peak": mpeak, "frac": values * 32 / t_s / 1e12 / mpeak}}
    return {"workload": "batched-64x16", "precision": prec, "systems": 64, "particles": total,
            "vectors": 16, "ms_per_step": ms, "targets_per_s": total / (ms * 1e-3),
            "target_vectors_per_s": 16 * total / (ms * 1e-3), "autotune_s": t_tune,
            "leaf_sizes": sorted(set(leaves)), "far_values": far_values,
            "near_values": near_values, "units": info["units"],
            "workgroups": info["workgroups"], "graph_captures": info["graph_captures"],
            "roofline": roof, "E_par_max_sampled": max(errs) if errs else None,
            "E_par_sample": "systems 0, 4, ..., 60; vectors 0, 5, 10, 15; 200 targets each"}


def run_sweep(args, dev):
    """Yukawa (kappa 0.5) on 2e6 Plummer-sphere particles: theta x n sweep, both paths.
    Errors against the FP64 oracle (treecode) on 1000 sampled targets."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    n = 2_000_000
    pos, q = inputs.plummer_sphere(n, inputs.config_seed(2))
    t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(q[0]).to(dev)
    smp = inputs.sample_indices(n, 1000, inputs.sample_seed(2))
    ds = None
    if not args.no_cpu:
        import oracle
        log("sweep: oracle direct sum on the 1000 sampled targets")
        ds = oracle.direct(pos[smp], pos, q[0], kernel=oracle.YUKAWA, kappa=0.5)
    rows = []
    for theta in (0.5, 0.7, 0.8):
        for deg in (4, 6, 8, 10):
            ref = None
            if not args.no_cpu:
                import oracle
                ref = oracle.Treecode(pos, pos, theta, deg, 2000, 2000).potential(
                    q[0], kernel=oracle.YUKAWA, kappa=0.5, sample=smp)
            for prec in ("fp64", "fp32_mixed"):
                # threads per target: the library's autotuner at leaf size 2000
                _, tpt, _ = bltc.autotune(t, t, candidates=(2000,), use_cache=False, full=True,
                                          theta=theta, degree=deg, kernel="yukawa", kappa=0.5,
                                          precision=prec)
                plan = bltc.Plan(t, t, theta=theta, degree=deg, leaf_size=2000, batch_size=2000,
                                 kernel="yukawa", kappa=0.5, precision=prec, threads_per_target=tpt)
                phi = plan.execute(qd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    plan.execute(qd, out=phi)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / args.steps
                row = {"theta": theta, "n": deg, "precision": prec, "ms": ms,
                       "targets_per_s": n / (ms * 1e-3), "threads_per_target": tpt}
                if ref is not None:
                    got = phi.cpu().numpy()[smp]
                    row["E_par"] = rel_l2(ref, got)
                    row["E_tc"] = rel_l2(ds, got)
                    row["oracle_E_tc"] = rel_l2(ds, ref)
                rows.append(row)
                log(f"sweep {row}")
    return {"workload": "yukawa-plummer-2M sweep", "rows": rows}


def matched_accuracy(rows, slack=1.1):
    """Time against error (eq. 16) of both paths: for every FP64 cell on the FP64
    frontier (no faster FP64 cell with a smaller E_tc), the fastest FP32-mixed cell
    whose E_tc is at most `slack` times that cell's, and the time ratio."""
    f64 = sorted((r for r in rows if r["precision"] == "fp64"), key=lambda r: r["ms"])
    mixed = [r for r in rows if r["precision"] == "fp32_mixed"]
    frontier, best = [], float("inf")
    for r in f64:
        if r["E_tc"] < best:
            frontier.append(r)
            best = r["E_tc"]
    out = []
    for r in frontier:
        cand = [m for m in mixed if m["E_tc"] <= slack * r["E_tc"] and m["E_par"] <= 1e-6]
        m = min(cand, key=lambda x: x["ms"], default=None)
        out.append({"E_tc_fp64": r["E_tc"], "fp64": (r["theta"], r["n"]), "fp64_ms": r["ms"],
                    "fp32_mixed": None if m is None else (m["theta"], m["n"]),
                    "mixed_ms": None if m is None else m["ms"],
                    "E_tc_mixed": None if m is None else m["E_tc"],
                    "speedup": None if m is None else r["ms"] / m["ms"]})
    return out


def run_accuracy(args, dev):
    """Time against error on the headline geometry (10^6 uniform, Coulomb,
    N_L = N_B = 2000): theta in {0.5, 0.7, 0.8, 0.9} x n in 3..10, both paths, threads
    per target from the library's autotuner; E_tc against the oracle's direct sum
    and E_par against the oracle treecode on the 1000 sampled targets (Sec. IV,
    Fig. 4); then the matched-accuracy comparison of the two paths."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    w = WORKLOADS["uniform-1M"]
    n = w["n"]
    pos, q = inputs.uniform_cube(n, inputs.config_seed(w["cfg"]))
    t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(q[0]).to(dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    smp = inputs.sample_indices(n, w["samples"], inputs.sample_seed(w["cfg"]))
    import oracle
    log("accuracy: oracle direct sum on the 1000 sampled targets")
    ds = oracle.direct(pos[smp], pos, q[0])
    rows = []
    for theta in args.thetas:
        for deg in args.degrees:
            oc = oracle.Treecode(pos, pos, theta, deg, w["leaf"], w["batch"])
            ref = oc.potential(q[0], sample=smp)
            del oc
            for prec in ("fp64", "fp32_mixed"):
                _, tpt, _ = bltc.autotune(t, t, candidates=(w["leaf"],), use_cache=False, full=True,
                                          theta=theta, degree=deg, precision=prec)
                plan = bltc.Plan(t, t, theta=theta, degree=deg, leaf_size=w["leaf"],
                                 batch_size=w["batch"], precision=prec, threads_per_target=tpt)
                for _ in range(max(1, args.warmup)):
                    plan.execute(qd, out=phi)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    plan.execute(qd, out=phi)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / args.steps
                got = phi.cpu().numpy()[smp]
                row = {"theta": theta, "n": deg, "precision": prec, "ms": ms,
                       "targets_per_s": n / (ms * 1e-3), "threads_per_target": tpt,
                       "E_par": rel_l2(ref, got), "E_tc": rel_l2(ds, got),
                       "oracle_E_tc": rel_l2(ds, ref)}
                rows.append(row)
                del plan
                log(f"accuracy {row}")
    return {"workload": f"uniform-1M accuracy sweep: N={n} uniform [-1,1]^3, coulomb, "
                        f"N_L=N_B={w['leaf']}, 1000 sampled targets",
            "rows": rows, "matched": matched_accuracy(rows)}


def run_large(args, dev):
    """1.28e8 particles uniform in [-1,1]^3, Coulomb, theta 0.7, n 8, N_L = N_B = 4000."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    n = args.large_n
    log(f"large: generating {n} particles")
    g = inputs.rng(inputs.config_seed(4))
    pos = g.uniform(-1.0, 1.0, size=(3, n))        # SoA directly (the same distribution)
    q = g.uniform(-1.0, 1.0, size=n)
    t = torch.from_numpy(pos).to(dev)
    qd = torch.from_numpy(q).to(dev)
    res = {"workload": f"uniform-{n}", "particles": n, "method": args.large_method}
    for prec in ("fp64", "fp32_mixed"):
        t0 = time.perf_counter()
        plan = bltc.Plan(t, t, theta=0.7, degree=8, leaf_size=4000, batch_size=4000, precision=prec,
                         method=args.large_method)
        t_plan = time.perf_counter() - t0
        st = plan.stats()
        log(f"large {prec}: plan {t_plan:.1f}s {st['batches']} batches")
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        plan.set_timing(True)
        plan.execute(qd, out=phi)
        ph = plan.phase_times()
        res[prec] = {"plan_s": t_plan, "phases_ms": ph, "targets_per_s": n / (ph["total"] * 1e-3),
                     "end_to_end_targets_per_s": n / (t_plan + ph["total"] * 1e-3),
                     "far_evals": st["far_evals"], "near_evals": st["near_evals"],
                     "mutual_pairs": st["mutual_pairs"], "mutual_pair_evals": st["mutual_pair_evals"],
                     "pair_rounds": st["pair_rounds"],
                     "pair_workspace_bytes": st["pair_workspace_bytes"],
                     "workspace_bytes": st["workspace_bytes"]}
        log(f"large {prec}: {ph}")
        if prec == "fp64":
            phi64 = phi.clone()
        else:
            res["mixed_vs_fp64_fullN"] = float(torch.sqrt(torch.sum((phi - phi64) ** 2) /
                                                          torch.sum(phi64 ** 2)).item())
            phim = phi
        del plan
    # errors on 10,000 sampled targets against the FP64 direct sum (eq. 16): the GPU
    # direct-sum kernel (bltc_direct, parity-checked against the oracle in the tests),
    # cross-checked against the CPU oracle's direct sum on 300 of the targets
    smp = inputs.sample_indices(n, 10_000, inputs.sample_seed(4))
    smp_d = torch.from_numpy(smp).to(dev)
    ts = t[:, smp_d].contiguous()
    t0 = time.perf_counter()
    ds = bltc.direct(ts, t, qd)
    torch.cuda.synchronize()
    res["gpu_direct_s"] = time.perf_counter() - t0
    ds = ds.cpu().numpy()
    g64 = phi64[smp_d].cpu().numpy()
    gm = phim[smp_d].cpu().numpy()
    res["E_tc_10000"] = {"fp64": rel_l2(ds, g64), "fp32_mixed": rel_l2(ds, gm)}
    log(f"large: E_tc on 10,000 targets {res['E_tc_10000']}")
    if not args.no_cpu:
        import oracle
        post = np.ascontiguousarray(pos.T)
        parts = []
        for c in range(3):
            sub = smp[100 * c:100 * (c + 1)]
            parts.append(oracle.direct(post[sub], post, q))
            log(f"large: oracle direct sum, targets {100 * c}..{100 * (c + 1)} done")
        od = np.concatenate(parts)
        res["gpu_direct_vs_oracle_direct_300"] = rel_l2(od, ds[:300])
        res["E_tc_oracle_300"] = {"fp64": rel_l2(od, g64[:300]), "fp32_mixed": rel_l2(od, gm[:300])}
        res["oracle_threads"] = oracle.max_threads()
        log(f"large: oracle cross-check {res['gpu_direct_vs_oracle_direct_300']:.3e}")
        # E_par: the oracle treecode (host tree and lists of the whole set; modified
        # charges of the clusters the sampled batches need) on the 10,000 targets
        log("large: oracle treecode: building the trees and lists on the host")
        oc = oracle.Treecode(post, post, 0.7, 8, 4000, 4000)
        log(f"large: oracle treecode: {oc.n_batches} batches, {oc.n_clusters} clusters "
            f"({oc.t_setup:.1f}s); modified charges and the sampled potentials")
        ref, times = oc.potential(q, sample=smp, return_times=True)
        del oc
        res["E_par_10000"] = {"fp64": rel_l2(ref, g64), "fp32_mixed": rel_l2(ref, gm)}
        res["oracle_E_tc_10000"] = rel_l2(ds, ref)
        res["oracle_treecode_s"] = times
        log(f"large: E_par on 10,000 targets {res['E_par_10000']}; oracle E_tc "
            f"{res['oracle_E_tc_10000']:.3e}")
    return res


def run_multi(args, dev):
    """The headline points (10^6 uniform, Coulomb, theta 0.7, n 8, N_L = N_B = 2000)
    with 16 charge vectors through one multi-vector plan (kernel values shared,
    contraction on the matrix cores), FP64 and FP32-mixed, beside the one-vector
    FP64 plan on the first vector: per-vector throughput at the same accuracy.
    Errors against the oracle's treecode on the sampled targets, vectors 0 and 15."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    w = WORKLOADS["uniform-1M"]
    n, m = w["n"], 16
    log(f"multi: generating {n} particles, {m} charge vectors")
    pos, q = inputs.uniform_cube(n, inputs.config_seed(w["cfg"]), m=m)
    t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    phi = torch.empty((m, n), dtype=torch.float64, device=dev)
    smp = inputs.sample_indices(n, w["samples"], inputs.sample_seed(w["cfg"]))
    kw = dict(theta=w["theta"], degree=w["degree"], leaf_size=w["leaf"], batch_size=w["batch"])
    res = {"workload": f"multi uniform-1M x{m}: N={n}, {m} charge vectors, coulomb, "
                       f"theta={w['theta']}, n={w['degree']}, N_L=N_B={w['leaf']}", "paths": {}}

    def timed(plan, qv, out):
        for _ in range(args.warmup):
            plan.execute(qv, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(qv, out=out)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps

    # the plain FP64 path: one vector per evaluation, its own autotuned lanes per target
    _, tpt, _ = bltc.autotune(t, t, candidates=(w["leaf"],), use_cache=False, full=True,
                              precision="fp64", **{k: v for k, v in kw.items()
                                                   if k in ("theta", "degree")})
    one = bltc.Plan(t, t, precision="fp64", threads_per_target=max(1, tpt), **kw)
    ms1 = timed(one, qd[0].contiguous(), phi[0])
    del one
    res["one_vector_fp64"] = {"ms_per_vector": ms1, "targets_per_s": n / (ms1 * 1e-3),
                              "threads_per_target": max(1, tpt)}
    log(f"multi: one-vector FP64 {ms1:.2f} ms per vector")
    got = {}
    for prec in ("fp64", "fp32_mixed"):
        plan = bltc.Plan(t, t, precision=prec, max_q=m, **kw)
        ms = timed(plan, qd, phi)
        got[prec] = phi[[0, m - 1]].cpu().numpy()
        res["paths"][prec] = {"ms_per_step": ms, "ms_per_vector": ms / m,
                              "target_vectors_per_s": m * n / (ms * 1e-3),
                              "speedup_per_vector_vs_one_vector_fp64": ms1 / (ms / m)}
        log(f"multi {prec}: {ms:.1f} ms for {m} vectors ({ms / m:.2f} ms per vector, "
            f"{ms1 / (ms / m):.2f}x the one-vector FP64 path)")
        del plan
    if not args.no_cpu:
        import oracle
        oc = oracle.Treecode(pos, pos, w["theta"], w["degree"], w["leaf"], w["batch"])
        ref = oc.potential(q[[0, m - 1]], sample=smp)
        for prec in got:
            res["paths"][prec]["E_par"] = max(rel_l2(ref[i], got[prec][i][smp]) for i in range(2))
            log(f"multi {prec}: E_par {res['paths'][prec]['E_par']:.2e} (vectors 0 and {m - 1})")
    return res


def run_variant(args, dev):
    """Cluster-particle (targets interpolated) or cluster-cluster (both sides)
    treecode on the headline workload: 10^6 uniform, Coulomb, theta 0.7, n 8,
    N_L = N_B = 2000, FP64 and FP32-mixed."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    w = WORKLOADS["uniform-1M"]
    n = w["n"]
    log(f"cp: generating {n} particles")
    pos, q = inputs.uniform_cube(n, inputs.config_seed(w["cfg"]))
    t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(q[0]).to(dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    smp = inputs.sample_indices(n, w["samples"], inputs.sample_seed(w["cfg"]))
    method = args.workload
    res = {"workload": f"{method} uniform-1M: N={n}, coulomb, theta={w['theta']}, n={w['degree']}, "
                       f"N_L=N_B={w['leaf']}", "paths": {}}
    got = {}
    for prec in ("fp64", "fp32_mixed"):
        t0 = time.perf_counter()
        plan = bltc.Plan(t, t, method=method, theta=w["theta"], degree=w["degree"],
                         leaf_size=w["leaf"], batch_size=w["batch"], precision=prec)
        t_plan = time.perf_counter() - t0
        st = plan.stats()
        for _ in range(args.warmup):
            plan.execute(qd, out=phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(qd, out=phi)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        plan.set_timing(True)
        plan.execute(qd, out=phi)
        ph = plan.phase_times()
        plan.set_timing(False)
        got[prec] = phi.cpu().numpy()
        res["paths"][prec] = {
            "ms_per_step": ms, "targets_per_s": n / (ms * 1e-3), "plan_s": t_plan,
            "end_to_end_targets_per_s": n / (t_plan + ms * 1e-3),
            "phases_ms": {"gather": ph["gather"], "proxy_potentials": ph["upward"],
                          "direct_and_interpolation": ph["interact"], "total": ph["total"]},
            "approx_evals": st["far_evals"], "near_evals": st["near_evals"],
            "interp_terms": st["upward_terms"],
            "approx_pairs": st["approx_pairs"], "direct_pairs": st["direct_pairs"],
            "mutual_pair_evals": st["mutual_pair_evals"]}
        # the interaction launches (proxy potentials, direct sums and, for the
        # cluster-cluster method, grid-grid and grid-targets pairs) are bound by
        # VALU issue; the phases also hold the small upward / interpolation work
        t_int = (ph["upward"] + ph["interact"]) * 1e-3
        mutual = st["mutual_pair_evals"]   # direct kernel values serving two terms
        ach = ((st["far_evals"] + st["near_evals"] - 2 * mutual) * FLOPS_COULOMB +
               mutual * FLOPS_MUTUAL_PAIR) / t_int / 1e12
        peak = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
        res["paths"][prec]["roofline"] = {
            "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "traffic": None, "kernel": "interact (proxy + targets launches)",
            "flops_per_eval": FLOPS_COULOMB}
        log(f"{method} {prec}: {ms:.2f} ms/step, phases {ph}")
        del plan
    if not args.no_cpu:
        import oracle
        cls = oracle.ClusterParticle if method == "cp" else oracle.ClusterCluster
        oc = cls(pos, pos, w["theta"], w["degree"], w["leaf"], w["batch"])
        ref, times = oc.potential(q[0], sample=smp, return_times=True)
        ds = oracle.direct(pos[smp], pos, q[0])
        for prec, v in got.items():
            res["paths"][prec]["E_par"] = rel_l2(ref, v[smp])
            res["paths"][prec]["E_tc"] = rel_l2(ds, v[smp])
        res["oracle_E_tc"] = rel_l2(ds, ref)
        # the oracle forms the proxy potentials (and modified charges) of every
        # cluster on the sampled paths (nearly all of them) and evaluates the
        # sample: extrapolate
        t_full = times["proxy"] + times["eval"] * n / len(smp)
        res["cpu_baseline"] = {"value": n / t_full, "unit": "targets/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"{len(smp)} sampled targets: proxy potentials "
                                         f"{times['proxy']:.1f}s + evaluation {times['eval']:.2f}s, "
                                         f"extrapolated to N"}
        log(f"{method}: errors {[(p, res['paths'][p]['E_par'], res['paths'][p]['E_tc']) for p in got]}")
    return res


def run_hermite(args, dev):
    """Barycentric Hermite treecode (FP64 and FP32-mixed) on the headline geometry:
    10^6 uniform, Coulomb, theta 0.7, N_L = N_B = 2000, degrees 2..4 (8 (n+1)^3 <= 1000
    modified charges per cluster, against 729 for the BLTC at n = 8)."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    w = WORKLOADS["uniform-1M"]
    n = w["n"]
    log(f"hermite: generating {n} particles")
    pos, q = inputs.uniform_cube(n, inputs.config_seed(w["cfg"]))
    t = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(q[0]).to(dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    smp = inputs.sample_indices(n, w["samples"], inputs.sample_seed(w["cfg"]))
    res = {"workload": f"hermite uniform-1M: N={n}, coulomb, theta={w['theta']}, "
                       f"N_L=N_B={w['leaf']}", "degrees": {}}
    got = {}
    for deg in args.hermite_degrees:
        res["degrees"][deg] = {}
        for prec in ("fp64", "fp32_mixed"):
            # threads per target: the library's autotuner at the workload's leaf size
            _, tpt, _ = bltc.autotune(t, t, candidates=(w["leaf"],), use_cache=False, full=True,
                                      method="hermite", theta=w["theta"], degree=deg,
                                      precision=prec)
            t0 = time.perf_counter()
            plan = bltc.Plan(t, t, method="hermite", theta=w["theta"], degree=deg,
                             leaf_size=w["leaf"], batch_size=w["batch"], precision=prec,
                             threads_per_target=tpt)
            t_plan = time.perf_counter() - t0
            st = plan.stats()
            for _ in range(args.warmup):
                plan.execute(qd, out=phi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                plan.execute(qd, out=phi)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            plan.set_timing(True)
            ph = {"gather": 0.0, "upward": 0.0, "interact": 0.0, "total": 0.0, "mutual_pairs": 0.0}
            for _ in range(args.steps):
                plan.execute(qd, out=phi)
                for k, v in plan.phase_times().items():
                    ph[k] += v / args.steps
            plan.set_timing(False)
            got[(deg, prec)] = phi.cpu().numpy()
            points = st["far_evals"] // 8      # far_evals counts 8 values per grid point
            mutual = st["mutual_pair_evals"]   # direct kernel values serving two terms
            flops = (points * FLOPS_HERMITE_POINT + (st["near_evals"] - 2 * mutual) * FLOPS_COULOMB +
                     mutual * FLOPS_MUTUAL_PAIR)
            ach = flops / (ph["interact"] * 1e-3) / 1e12
            peak = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
            kern = "f64" if prec == "fp64" else "mixed"
            res["degrees"][deg][prec] = {
                "ms_per_step": ms, "targets_per_s": n / (ms * 1e-3), "plan_s": t_plan,
                "threads_per_target": tpt,
                "phases_ms": ph, "grid_point_evals": points, "near_evals": st["near_evals"],
                "mutual_pair_evals": mutual,
                "approx_pairs": st["approx_pairs"], "direct_pairs": st["direct_pairs"],
                "roofline": {"bound": "alu", "achieved": ach, "peak": peak,
                             "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                             "kernel": f"interaction phase: interact_hermite_{kern}<{deg}, 0> + "
                                       f"near_pairs_{kern}<0>",
                             "flops_per_grid_point": FLOPS_HERMITE_POINT,
                             "flops_per_near_eval": FLOPS_COULOMB}}
            log(f"hermite n={deg} {prec}: {ms:.2f} ms/step, phases {ph}")
            del plan
    if not args.no_cpu:
        import oracle
        ds = oracle.direct(pos[smp], pos, q[0])
        for deg in args.hermite_degrees:
            oc = oracle.Treecode(pos, pos, w["theta"], deg, w["leaf"], w["batch"], hermite=True)
            ref, times = oc.potential(q[0], sample=smp, return_times=True)
            for prec in ("fp64", "fp32_mixed"):
                v = got[(deg, prec)]
                r = res["degrees"][deg][prec]
                r["E_par"] = rel_l2(ref, v[smp])
                r["E_tc"] = rel_l2(ds, v[smp])
                log(f"hermite n={deg} {prec}: E_par {r['E_par']:.2e} E_tc {r['E_tc']:.2e}")
            res["degrees"][deg]["oracle_s"] = times
    return res


def run_setup(args, dev):
    """Setup phase alone: plans built on the GPU (device coordinates) against the
    host planner (host coordinates) on the same uniform cube, N_L = N_B = 4000."""
    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    n = args.large_n
    log(f"setup: generating {n} particles")
    g = inputs.rng(inputs.config_seed(4))
    pos = g.uniform(-1.0, 1.0, size=(3, n))
    t = torch.from_numpy(pos).to(dev)
    kw = dict(theta=0.7, degree=8, leaf_size=4000, batch_size=4000)
    res = {"workload": f"setup uniform-{n}", "particles": n}
    for prec in ("fp64", "fp32_mixed"):
        times = []
        for rep in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = bltc.Plan(t, t, precision=prec, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            st = plan.stats()
            del plan
            log(f"setup {prec}: device plan {times[-1]:.3f}s")
        res[prec] = {"device_plan_s": min(times), "device_plan_s_all": times,
                     "clusters": st["clusters"], "batches": st["batches"],
                     "approx_pairs": st["approx_pairs"], "direct_pairs": st["direct_pairs"],
            "mutual_pair_evals": st["mutual_pair_evals"]}
    if n <= args.setup_host_max:
        ph = np.ascontiguousarray(pos)
        t0 = time.perf_counter()
        hplan = bltc.Plan(ph, ph, host=True, **kw)
        res["host_plan_s"] = time.perf_counter() - t0
        log(f"setup: host plan {res['host_plan_s']:.3f}s")
        del hplan
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform-1M",
                    choices=sorted(WORKLOADS) + ["batched-64x16", "yukawa-plummer-sweep", "uniform-large",
                                                 "setup", "cp", "cc", "hermite", "accuracy-sweep",
                                                 "multi-1M"])
    ap.add_argument("--thetas", type=float, nargs="+", default=[0.5, 0.7, 0.8, 0.9],
                    help="accuracy-sweep workload: MAC parameters")
    ap.add_argument("--degrees", type=int, nargs="+", default=[3, 4, 5, 6, 7, 8, 9, 10],
                    help="accuracy-sweep workload: interpolation degrees")
    ap.add_argument("--large-n", type=int, default=128_000_000)
    ap.add_argument("--large-method", default="bltc", choices=["bltc", "cp", "cc"],
                    help="uniform-large workload: treecode variant")
    ap.add_argument("--hermite-degrees", type=int, nargs="+", default=[2, 3, 4],
                    help="hermite workload: interpolation degrees")
    ap.add_argument("--setup-host-max", type=int, default=20_000_000,
                    help="setup workload: also time the host planner up to this many particles")
    ap.add_argument("--precision", default="both", choices=["fp64", "fp32_mixed", "both"])
    ap.add_argument("--threads-per-target", type=int, default=0, choices=[0, 1, 2, 4],
                    help="headline workloads: lanes per target (0: the library's autotuner "
                         "picks 1, 2 or 4 at the workload's leaf size)")
    ap.add_argument("--cpu-sample", type=int, default=150000,
                    help="targets the CPU oracle evaluates for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (no errors, no CPU baseline)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2003_01836_amd as bltc
    from paper_2003_01836_amd import inputs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if args.workload in ("batched-64x16", "yukawa-plummer-sweep", "uniform-large", "setup", "cp",
                         "cc", "hermite", "accuracy-sweep", "multi-1M"):
        fn = {"batched-64x16": run_batched, "yukawa-plummer-sweep": run_sweep,
              "uniform-large": run_large, "setup": run_setup, "cp": run_variant,
              "cc": run_variant, "hermite": run_hermite,
              "accuracy-sweep": run_accuracy, "multi-1M": run_multi}[args.workload]
        print(json.dumps(fn(args, dev)), flush=True)
        return 0
    w = WORKLOADS[args.workload]
    n = w["n"]
    log(f"workload {args.workload}: generating {n} particles")
    pos, q = inputs.uniform_cube(n, inputs.config_seed(w["cfg"]))
    t_soa = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    qd = torch.from_numpy(q[0]).to(dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    smp = inputs.sample_indices(n, w["samples"], inputs.sample_seed(w["cfg"]))

    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written")
        del a, b

    precisions = ["fp64", "fp32_mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precisions:
        tpt = args.threads_per_target
        if tpt == 0 and w["leaf"] == w["batch"]:
            # threads per target: the library's autotuner at the workload's leaf size
            _, tpt, tune_ms = bltc.autotune(t_soa, t_soa, candidates=(w["leaf"],), use_cache=False,
                                            full=True, theta=w["theta"], degree=w["degree"],
                                            kernel=w["kernel"], kappa=w["kappa"], precision=prec)
            log(f"{prec}: autotuner: {tpt} threads per target ({tune_ms:.2f} ms)")
        tpt = max(1, tpt)
        log(f"{prec}: planning")
        t0 = time.perf_counter()
        plan = bltc.Plan(t_soa, t_soa, theta=w["theta"], degree=w["degree"], leaf_size=w["leaf"],
                         batch_size=w["batch"], kernel=w["kernel"], kappa=w["kappa"], precision=prec,
                         threads_per_target=tpt)
        t_plan = time.perf_counter() - t0
        st = plan.stats()
        log(f"{prec}: plan {t_plan:.2f}s, {st['batches']} batches, {st['approx_pairs']} approx + "
            f"{st['direct_pairs']} direct pairs")
        for _ in range(args.warmup):
            plan.execute(qd, out=phi)
        torch.cuda.synchronize()
        log(f"{prec}: warmup done; timing {args.steps} steps")
        # the timed steps record HIP events between the phases on the plan's
        # stream (bltc_plan_set_timing); each step's phase times are read after it
        plan.set_timing(True)
        ph = {"gather": 0.0, "upward": 0.0, "interact": 0.0, "total": 0.0, "mutual_pairs": 0.0}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(qd, out=phi)
            for k, v in plan.phase_times().items():
                ph[k] += v / args.steps
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t0
        plan.set_timing(False)
        ms_step = 1e3 * t_total / args.steps
        got = phi.cpu().numpy()
        log(f"{prec}: {ms_step:.3f} ms/step; phases {ph}")
        results[prec] = dict(plan=plan, stats=st, ms=ms_step, phases=ph, phi=got, t_plan=t_plan,
                             tpt=tpt)

    cpu = None
    errors = {}
    if not args.no_cpu:
        import oracle
        log("oracle: building tree and lists on the host")
        oc = oracle.Treecode(pos, pos, w["theta"], w["degree"], w["leaf"], w["batch"])
        kern = oracle.YUKAWA if w["kernel"] == "yukawa" else oracle.COULOMB
        ref, times = oc.potential(q[0], kernel=kern, kappa=w["kappa"], sample=smp, return_times=True)
        log("oracle: direct sum on the sample")
        ds = oracle.direct(pos[smp], pos, q[0], kernel=kern, kappa=w["kappa"])
        for prec, r in results.items():
            errors[prec] = {"E_par": rel_l2(ref, r["phi"][smp]), "E_tc": rel_l2(ds, r["phi"][smp])}
        errors["oracle"] = {"E_tc": rel_l2(ds, ref)}
        # CPU baseline: the oracle's evaluation phase on a bounded sample
        cs = inputs.sample_indices(n, min(args.cpu_sample, n), inputs.sample_seed(w["cfg"]) + 1)
        log(f"oracle: timing the CPU baseline on {len(cs)} targets")
        _, ctimes = oc.potential(q[0], kernel=kern, kappa=w["kappa"], sample=cs, return_times=True)
        t_cpu = ctimes["upward"] + ctimes["eval"]
        cpu = {"value": len(cs) / t_cpu, "unit": "targets/s", "cores": oracle.max_threads(),
               "cpu_model": cpu_model(),
               "kind": "oracle",
               "sample": (f"{len(cs)} sampled targets of the same plan: tree/lists built once "
                          f"({oc.t_setup:.2f}s, excluded); modified charges for every cluster their "
                          f"batches need ({ctimes['upward']:.2f}s) + evaluation ({ctimes['eval']:.2f}s)")}
        log(f"oracle: {cpu['value']:.1f} targets/s on {cpu['cores']} threads")

    # headline: the FP64 path, the paper's precision (Sec. IV); the FP32-mixed path
    # is reported beside it with its own roofline and the equal-accuracy test
    head = "fp64" if "fp64" in results else precisions[0]
    r = results[head]
    st = r["stats"]
    ker_id = 1 if w["kernel"] == "yukawa" else 0
    trans_per_eval = 2 if w["kernel"] == "yukawa" else 1
    flops_eval = FLOPS_YUKAWA if w["kernel"] == "yukawa" else FLOPS_COULOMB

    def path_roofline(prec, v):
        """Roofline of one path's interaction launches: the pair kernel (kernel values
        = mutual_pair_evals, each serving two direct terms) and the batch kernel (far
        field, the other direct terms), each from its HIP-event time in the timed steps."""
        sv = v["stats"]
        evals = sv["far_evals"] + sv["near_evals"]
        mutual = sv.get("mutual_pair_evals", 0)
        t_pairs = v["phases"].get("mutual_pairs", 0.0)
        t_batch = v["phases"]["interact"] - t_pairs
        suffix = "f64" if prec == "fp64" else "mixed"
        peak = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
        kernels = {f"interact_{suffix}": {"evals": evals - 2 * mutual, "flops_per_eval": flops_eval,
                                          "ms_per_launch": t_batch}}
        if mutual:
            kernels[f"near_pairs_{suffix}"] = {"evals": mutual,
                                               "flops_per_eval": flops_eval + FLOPS_PAIR_EXTRA,
                                               "ms_per_launch": t_pairs}
        for kn, kv in kernels.items():
            kv["achieved"] = kv["evals"] * kv["flops_per_eval"] / (kv["ms_per_launch"] * 1e-3) / 1e12
            kv["frac"] = kv["achieved"] / peak
            # the pair kernel does not depend on the threads per target
            kt = v["tpt"] if kn.startswith("interact") else 1
            kv["traffic"] = counter_traffic(kn, w["degree"], ker_id, kt)
            kv["issue"] = issue_model(kn, w["degree"], ker_id, trans_per_eval, kv["evals"],
                                      kv["ms_per_launch"], kt)
        kname = max(kernels, key=lambda k: kernels[k]["ms_per_launch"])
        kd = kernels[kname]
        phase_flops = sum(x["evals"] * x["flops_per_eval"] for x in kernels.values())
        phase_achieved = phase_flops / (v["phases"]["interact"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": kd["achieved"], "peak": peak, "unit": "TFLOP/s",
                "frac": kd["frac"], "traffic": kd["traffic"],
                "kernel": kname, "flops_per_eval": kd["flops_per_eval"],
                "evals_per_launch": kd["evals"], "ms_per_launch": kd["ms_per_launch"],
                "issue": kd["issue"],
                "interaction_kernels": kernels,
                "interaction_phase": {"achieved": phase_achieved, "frac": phase_achieved / peak,
                                      "ms": v["phases"]["interact"]},
                "upward": upward_roofline(w["degree"], sv["upward_terms"], v["phases"]["upward"],
                                          prec)}

    paths = {}
    for p, v in results.items():
        ev = v["stats"]["far_evals"] + v["stats"]["near_evals"]
        paths[p] = {"targets_per_s": n / (v["ms"] * 1e-3), "ms_per_step": v["ms"],
                    "threads_per_target": v["tpt"], "phases_ms": v["phases"], "plan_s": v["t_plan"],
                    "end_to_end_targets_per_s": n / (v["t_plan"] + v["ms"] * 1e-3),
                    "terms_per_s": ev / (v["phases"]["interact"] * 1e-3),
                    **errors.get(p, {})}
        if p != head:
            paths[p]["roofline"] = path_roofline(p, v)
    if "fp64" in errors and "fp32_mixed" in errors:
        e64, emx = errors["fp64"], errors["fp32_mixed"]
        ratio = emx["E_tc"] / e64["E_tc"]
        paths["fp32_mixed"]["E_tc_ratio_to_fp64"] = ratio
        # equal accuracy: both paths within 1e-6 of the oracle treecode, and the
        # mixed path's error against the direct sum at most 1.1 x the FP64 path's
        paths["fp32_mixed"]["equal_accuracy"] = bool(e64["E_par"] <= 1e-6 and emx["E_par"] <= 1e-6
                                                     and ratio <= 1.1)
        paths["fp32_mixed"]["speedup_vs_fp64"] = results["fp64"]["ms"] / results["fp32_mixed"]["ms"]
    valid = head not in errors or errors[head]["E_par"] <= 1e-6
    line = {
        "metric": "targets/s at rel-L2 err <=1e-6 (BLTC evaluation phase)",
        "value": n / (r["ms"] * 1e-3) if valid else None,
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32-mixed",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={n} uniform [-1,1]^3, charges U[-1,1], "
                               f"{w['kernel']}, theta={w['theta']}, n={w['degree']}, "
                               f"N_L=N_B={w['leaf']}", "path": head,
                   "threads_per_target": r["tpt"]},
        "roofline": path_roofline(head, r),
        "cpu_baseline": cpu,
        "paths": paths,
        "oracle_E_tc": errors.get("oracle", {}).get("E_tc"),
        "stats": {k: st[k] for k in ("clusters", "batches", "approx_pairs", "direct_pairs",
                                     "far_evals", "near_evals", "upward_terms", "depth",
                                     "mutual_pair_evals")},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
