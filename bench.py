#!/usr/bin/env python3
"""Benchmark of the CFUST EM hot path on one MI355X.

One step = one EM iteration of the mixture of canonical fundamental skew t
distributions: the E-step (Sec. 3.1 of Lee, Leemaqz & McLachlan; lattice
estimates of T_q, T_{q-1}, T_{q-2}, moment assembly, log-sum-exp and the
log-likelihood, eqs. 4, 12-17, 27) followed by the M-step (Sec. 3.2, eqs.
18-22), both through the C ABI of libcfust.so.  Inputs are resident in HBM
before timing starts.

Workload (default): n = 20000 observations, p = q = 4, g = 3 components,
lattice N = 4096 points x S = 8 shifts, FP32 lattice integrand with FP64
elsewhere; synthetic data drawn from the model's hierarchy (eq. 6).

Prints one JSON line with the throughput in (observation x component) pairs
per second, the roofline position of the lattice kernels (FP32 VALU), and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CFUST E-step (obs×comp)/s at stated tol vs FP64 oracle; surrogate vs QMC speedup"
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (chip figure: 2 wave64 FMA issues per CU per cycle)

# Kernel sources that the measured constants below belong to: the FP32
# operations per lattice point and the HBM bytes of the lattice kernels were
# read from rocprofv3 counters for sources with this digest; when the sources
# change, the bench reports those figures as null until they are measured
# again (profiles/k_estep_qmc_counters.md).
TRAFFIC_SOURCES = ["paper_1606_02054_amd/csrc/cfust_sov.h", "paper_1606_02054_amd/csrc/cfust_devmath.h",
                   "paper_1606_02054_amd/csrc/cfust_estep.hip", "paper_1606_02054_amd/csrc/cfust_common.h"]
KERNEL_DIGEST = "f55a6781832900f4"
# FP32 arithmetic of one lattice point of the m-variate integrand in the FP32
# lattice kernel: (2 x SQ_INSTS_VALU_FMA_F32 + MUL_F32 + ADD_F32 + TRANS_F32)
# of a launch divided by the lattice points it evaluates.
LATTICE_FLOPS_PER_POINT = {2: 39.49, 3: 83.95, 4: 129.98, 5: 177.69, 6: 227.78, 7: 279.78, 8: 333.81}
# VALU issue of each kernel from SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU2 and
# GRBM_GUI_ACTIVE: wave64 VALU instructions per CU per cycle (the chip issues
# at most 2: one pair per SIMD per 4-cycle slot) and the share of them issued
# in pairs.
LATTICE_VALU_ISSUE = {
    2: {'valu_per_point': 39.1, 'valu_per_cu_cycle': 0.960, 'dual_issue_frac': 0.482, 'valu_slot_busy': 0.868},
    3: {'valu_per_point': 80.6, 'valu_per_cu_cycle': 1.084, 'dual_issue_frac': 0.558, 'valu_slot_busy': 0.941},
    4: {'valu_per_point': 122.8, 'valu_per_cu_cycle': 1.056, 'dual_issue_frac': 0.520, 'valu_slot_busy': 0.936},
    5: {'valu_per_point': 165.3, 'valu_per_cu_cycle': 0.991, 'dual_issue_frac': 0.487, 'valu_slot_busy': 0.893},
    6: {'valu_per_point': 210.7, 'valu_per_cu_cycle': 1.112, 'dual_issue_frac': 0.533, 'valu_slot_busy': 0.973},
    7: {'valu_per_point': 256.0, 'valu_per_cu_cycle': 1.039, 'dual_issue_frac': 0.473, 'valu_slot_busy': 0.939},
    8: {'valu_per_point': 301.9, 'valu_per_cu_cycle': 0.984, 'dual_issue_frac': 0.469, 'valu_slot_busy': 0.891},
}
# HBM bytes per launch of the FP32 lattice kernel of each dimension at the
# default workload (MiB read, MiB written: FETCH_SIZE x 2 and WRITE_SIZE x 1 in
# KiB, the factors that a 1 GiB device copy gives these counters).
TRAFFIC_MIB = {4: (2 * 12222.8 / 1024, 8080.4 / 1024), 3: (2 * 5074.0 / 1024, 6518.6 / 1024),
               2: (2 * 4029.0 / 1024, 7761.2 / 1024)}


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_current() -> bool:
    return kernel_digest() == KERNEL_DIGEST


def lattice_flops_per_point(m: int):
    """Counter-measured FP32 flops of one lattice point of an m-variate T_m
    (None when the kernel sources changed since the counters were taken)."""
    if not counters_current():
        return None
    return LATTICE_FLOPS_PER_POINT.get(m)


def integral_dims(q: int):
    dims = [q, q] + [q - 1] * q + [q - 2] * (q * (q - 1) // 2)
    return [m for m in dims if m >= 2]


def lattice_roofline(prof, points_by_m, steps: int, kernel: str, traffic=None) -> dict:
    """Roofline of the FP32 lattice kernels from the HIP events that bracket
    them (prof: {m: (total ms, launches)} over `steps` steps) and the lattice
    points each dimension evaluates per step.  The top level is the dominant
    kernel (the dimension with the most time); `all_lattice` aggregates every
    dimension."""
    per = {}
    for m in sorted(prof):
        if m not in points_by_m or prof[m][1] == 0:
            continue
        ms_launch = prof[m][0] / prof[m][1]
        launches = prof[m][1] / steps
        fpp = lattice_flops_per_point(m)
        flops = fpp * points_by_m[m] / launches if fpp is not None else None
        per[m] = {"avg_ms": ms_launch, "launches_per_step": launches, "points_per_launch": points_by_m[m] / launches,
                  "flops_per_point": fpp, "achieved": flops / (ms_launch / 1e3) / 1e12 if flops else None,
                  "valu_issue": LATTICE_VALU_ISSUE.get(m) if counters_current() else None}
    if not per:
        return {"bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": traffic, "kernel": kernel}
    dom = max(per, key=lambda m: per[m]["avg_ms"] * per[m]["launches_per_step"])
    d = per[dom]
    tot_ms = sum(v["avg_ms"] * v["launches_per_step"] for v in per.values())
    tot_f = None
    if all(v["flops_per_point"] is not None for v in per.values()):
        tot_f = sum(v["flops_per_point"] * v["points_per_launch"] * v["launches_per_step"] for v in per.values())
    tr = None
    if traffic and dom in traffic:
        rd, wr = traffic[dom]
        tr = (rd + wr) * (1 << 20)
    return {"bound": "alu", "achieved": d["achieved"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": d["achieved"] / PEAK_FP32_TFLOPS if d["achieved"] else None, "traffic": tr,
            "traffic_MiB_read_write_per_launch": {f"m{m}": v for m, v in traffic.items()} if traffic else None,
            "kernel": f"{kernel}, m = {dom} (the dimension with the most time)",
            "flops_per_launch": d["flops_per_point"] * d["points_per_launch"] if d["flops_per_point"] else None,
            "avg_launch_ms": d["avg_ms"], "valu_issue": d["valu_issue"],
            "all_lattice": {"ms_per_step": tot_ms, "achieved": tot_f / (tot_ms / 1e3) / 1e12 if tot_f else None,
                            "frac": tot_f / (tot_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS if tot_f else None},
            "per_kernel": {f"m{m}": v for m, v in per.items()}}


def surrogate_vs_lattice(cf, ds, y, params, design, pairs):
    """E-step with the trained networks (T_m, m = 2..4, lattice fallback) against
    the plain lattice E-step at several lattice sizes, both measured by their
    log-likelihood error against a 4x larger lattice; speed-up at equal accuracy."""
    import torch
    from paper_1606_02054_amd import surrogate as S
    from cfust_inputs import make_design
    wdir = os.path.join(ROOT, "paper_1606_02054_amd", "weights")
    models = {}
    for m in (2, 3, 4):
        f = os.path.join(wdir, f"surrogate_m{m}.npz")
        if os.path.exists(f):
            models[m] = S.SurrogateNet.load(f)
    if not models:
        return {"skipped": "no trained weights under paper_1606_02054_amd/weights"}

    def timed(fn, reps=3):
        o = fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            o = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3, float(o.loglik.cpu()[0])

    ref_q = cf.device_qmc(make_design(4 * design.N, 2 * design.S, seed=4242), cf.CFUST_MIXED)
    ref = cf.cfust_estep(y, params, ref_q)
    torch.cuda.synchronize()
    l_ref = float(ref.loglik.cpu()[0])
    lat = []
    for N, Sh in [(128, 2), (256, 4), (512, 4), (1024, 4), (2048, 8), (design.N, design.S)]:
        q = cf.device_qmc(make_design(N, Sh, seed=1606), cf.CFUST_MIXED)
        ms, ll = timed(lambda: cf.cfust_estep(y, params, q))
        lat.append({"N": N, "S": Sh, "ms": ms, "abs_dloglik": abs(ll - l_ref)})
    q0 = cf.device_qmc(design, cf.CFUST_MIXED)
    sur = []
    for tol in (0.02, 0.05, 0.1):
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        ms, ll = timed(lambda: S.cfust_estep_surrogate(y, params, q0, models, tol, n_fallback=nf))
        J = len(integral_dims(params.q))
        err = abs(ll - l_ref)
        ok = [r for r in lat if r["abs_dloglik"] <= err]
        eq = min(ok, key=lambda r: r["ms"]) if ok else None
        sur.append({"tol": tol, "ms": ms, "abs_dloglik": err, "fallback_frac": int(nf.cpu()[0]) / (pairs * J),
                    "lattice_at_equal_accuracy": eq and {"N": eq["N"], "S": eq["S"], "ms": eq["ms"]},
                    "speedup_at_equal_accuracy": (eq["ms"] / ms) if eq else None})
    return {"reference": {"N": 4 * design.N, "S": 2 * design.S, "loglik": l_ref}, "lattice": lat,
            "surrogate": sur, "models": sorted(models)}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix


def _event_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def component_rooflines(cf, dev) -> dict:
    """The other bound kernels of the path, each against its own roofline:
    the M-step reduction (HBM) at the cytometry shape n = 1e6, p = q = 8,
    g = 5 with mixed-precision E-step arrays (values synthetic: the reduction
    reads every input once whatever it holds), and the surrogate network's
    BF16 matrix kernels (forward, and forward + backward of a training step)."""
    import numpy as np
    import torch
    from cfust_inputs.synth import draw_params
    from paper_1606_02054_amd import surrogate as S
    from paper_1606_02054_amd._binding import MLP_K, MLP_N

    out = {}
    n, p, q, g = 1_000_000, 8, 8, 5
    gen = torch.Generator(device=dev).manual_seed(5)
    y = torch.rand((p, n), dtype=torch.float64, device=dev, generator=gen) * 1024.0
    es = cf.alloc_estep(n, p, q, g, cf.CFUST_MIXED, device=dev, logf_comp=False, stderr=False)
    es.tau.copy_(torch.rand((g, n), dtype=torch.float64, device=dev, generator=gen))
    for t in (es.w, es.e1, es.e2, es.e3):
        t.copy_(torch.rand(t.shape, dtype=torch.float32, device=dev, generator=gen))
    P = cf.device_params(draw_params(np.random.default_rng(3), p, q, g, sigma="wishart"), device=dev)
    nxt = P.clone()
    ms = _event_ms(lambda: cf.cfust_mstep(y, es, P, out=nxt), 5)
    byts = n * (g * (8 + 4 * (2 + q + q * (q + 1) // 2)) + 8 * p)
    out["mstep"] = {"bound": "hbm", "kernel": "k_mstep_reduce + k_mstep_solve (cfust_mstep)",
                    "config": {"n": n, "p": p, "q": q, "g": g, "precision": "mixed"},
                    "ms": ms, "algorithmic_bytes": byts, "achieved": byts / (ms / 1e3) / 1e9,
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": byts / (ms / 1e3) / 1e9 / PEAK_HBM_GBS}
    del y, es
    net = S.SurrogateNet(3, seed=1, device=dev)
    B = 65536
    X0 = torch.zeros((B, 16), dtype=torch.int16, device=dev)
    o = torch.zeros((B, 16), dtype=torch.float32, device=dev)
    acts = S.Activations(B, dev)
    kn = sum(k * nn for k, nn in zip(MLP_K, MLP_N))
    f_fwd = 2.0 * B * kn
    ms_f = _event_ms(lambda: S.mlp_forward(net, X0, o), 10)          # inference: fused kernel
    dout = torch.zeros_like(o)
    ms_fb = _event_ms(lambda: (S.mlp_forward(net, X0, o, acts), S.mlp_backward(net, acts, dout)), 10)
    f_bwd = 2.0 * B * kn + 2.0 * B * (kn - MLP_K[0] * MLP_N[0])
    out["surrogate_forward"] = {"bound": "mfma", "kernel": "k_mlp_fwd_fused (inference, 16-4x256-16, B=65536)",
                                "ms": ms_f, "achieved": f_fwd / (ms_f / 1e3) / 1e12, "peak": PEAK_BF16_TFLOPS,
                                "unit": "TFLOP/s", "frac": f_fwd / (ms_f / 1e3) / 1e12 / PEAK_BF16_TFLOPS}
    tb = train_step_bytes(B)
    out["surrogate_train_step"] = {"bound": "hbm",
                                   "kernel": "k_gemm_bf16 + k_act_back + k_col_sum + k_sum_split (forward with saved "
                                             "activations + backward, B=65536)",
                                   "ms": ms_fb, "algorithmic_bytes": tb, "achieved": tb / (ms_fb / 1e3) / 1e9,
                                   "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": tb / (ms_fb / 1e3) / 1e9 / PEAK_HBM_GBS,
                                   "mfma_tflops": (f_fwd + f_bwd) / (ms_fb / 1e3) / 1e12}
    return out


def train_step_bytes(B: int, nsplit: int = 16) -> int:
    """Bytes one training step of the network must move, each array once: the
    forward pass reads every layer input (BF16) and writes the FP32
    pre-activations and the BF16 activations in both layouts (kept for the
    backward pass); the backward pass reads dY (FP32) and Z, writes dZ in both
    BF16 layouts, sums dZ per column for the bias gradient, forms dW from dZ^T
    and X^T in nsplit batch slices (partials written and summed) and dX = dZ W
    into dY.  Weights (BF16) count once per product."""
    from paper_1606_02054_amd._binding import MLP_K, MLP_N
    L = len(MLP_K)
    tot = 0
    for l, (K, N) in enumerate(zip(MLP_K, MLP_N)):
        last = l == L - 1
        tot += B * K * 2 + N * K * 2                                   # forward: X_l, W_l
        tot += B * N * 4 if last else B * N * (4 + 2 + 2)              # out, or Z_l + X_{l+1} + X_{l+1}^T
        tot += B * N * 4 + (0 if last else B * N * 4)                  # backward: dY, Z_l
        tot += B * N * 2 * 2                                           # dZ, dZ^T written
        tot += B * N * 2                                               # column sums read dZ^T
        tot += B * N * 2 + B * K * 2 + nsplit * N * K * 4 * 2 + N * K * 4   # dW: dZ^T, X^T, partials, dW
        if l > 0:
            tot += B * N * 2 + N * K * 2 + B * K * 4                   # dX: dZ, W^T, dY written
    return tot


def initialisation(cf, ds, y, qmc, dev, nstarts: int = 8) -> dict:
    """Algorithm 1 on the bench data: nstarts k-means partitions (seeded
    input, computed on the host and not timed) x 9 values of alpha, every
    candidate's log-likelihood in one density-only batch."""
    import numpy as np
    import torch
    from cfust_inputs import kmeans_partitions

    g, q = ds.params.g, ds.params.q
    labels = torch.as_tensor(kmeans_partitions(ds.y, g, nstarts, seed=5), device=dev)
    cf.initialise(y, g, q, labels, qmc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ll, k = cf.initialise(y, g, q, labels, qmc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    llv = ll.cpu().numpy()
    n = int(y.shape[1])
    return {"starts": nstarts, "alphas": 9, "candidates": nstarts * 9, "valid": int(np.isfinite(llv).sum()),
            "ms": ms, "candidate_pairs_per_s": nstarts * 9 * n * g / (ms / 1e3), "best_index": k,
            "best_loglik": float(llv.ravel()[k]) if k >= 0 else None}


def host_cpu() -> dict:
    """Model name and logical CPU count of the host (for the CPU baseline)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def progress(msg: str) -> None:
    """One line on stderr per finished bench section (stdout carries only the
    JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def precision_split(cf, y, params, design, dev, rows: int = 1024) -> dict:
    """One E-step over the first ``rows`` observations of the bench workload in
    mixed precision (FP32 lattice integrand) and in FP64 throughout, on the same
    lattice: the time of each and the largest difference of the
    per-observation log-density.  The FP64 path evaluates every t CDF by a
    continued fraction and every quantile by a root search, so it is timed on
    a slice of the data."""
    import torch
    ys = y[:, :rows].contiguous()
    out = {"rows": int(ys.shape[1])}
    res = {}
    for name, prec in (("mixed", cf.CFUST_MIXED), ("fp64", cf.CFUST_FP64)):
        qmc = cf.device_qmc(design, prec, device=dev)
        cf.cfust_estep(ys[:, :64].contiguous(), params, qmc)       # allocations, tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es = cf.cfust_estep(ys, params, qmc)
        torch.cuda.synchronize()
        out[f"{name}_estep_ms"] = (time.perf_counter() - t0) * 1e3
        res[name] = es.logf_obs.cpu().numpy()
        progress(f"precision split: {name} E-step over {rows} rows {out[name + '_estep_ms']:.1f} ms")
    out["fp64_over_mixed_time"] = out["fp64_estep_ms"] / out["mixed_estep_ms"]
    out["max_abs_dlogf_obs"] = float(abs(res["mixed"] - res["fp64"]).max())
    return out


def small_fit(cf, dev, nstarts: int = 4, iters: int = 20) -> dict:
    """The small configuration end to end in FP64: n = 1000, p = q = 2, g = 2,
    lattice 1024 x 4; Algorithm 1 over nstarts k-means partitions (seeded
    input, computed on the host and not timed) x 9 values of alpha, then
    iters EM iterations."""
    import torch
    from cfust_inputs import kmeans_partitions, make_design, workload
    ds = workload("cfust_n1000_p2_q2_g2")
    g, q = ds.params.g, ds.params.q
    y = torch.as_tensor(ds.y_soa, device=dev)
    qmc = cf.device_qmc(make_design(ds.meta["N"], ds.meta["S"], seed=1606), cf.CFUST_FP64, device=dev)
    labels = torch.as_tensor(kmeans_partitions(ds.y, g, nstarts, seed=7), device=dev)
    cf.initialise(y, g, q, labels, qmc)                # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params, ll0, k = cf.initialise(y, g, q, labels, qmc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(iters):
        es = cf.cfust_estep(y, params, qmc)
        params = cf.cfust_mstep(y, es, params)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"n": int(ds.y.shape[0]), "p": int(ds.y.shape[1]), "q": q, "g": g, "N": ds.meta["N"],
            "S": ds.meta["S"], "precision": "fp64", "starts": nstarts, "alphas": 9,
            "init_ms": (t1 - t0) * 1e3, "em_ms_per_iteration": (t2 - t1) * 1e3 / iters, "iterations": iters,
            "loglik_start": float(ll0.cpu().numpy().ravel()[k]), "loglik_end": float(es.loglik.cpu()[0])}


def small_restarts(cf, h, prec, dev, nstarts: int = 64, iters: int = 5) -> dict:
    """64 restarts of EM on the same n = 1000, p = q = 2, g = 2 data (the
    starts of Algorithm 1), lattice 1024 x 4: one batched EM iteration of all
    of them against the same starts run one after the other."""
    import torch
    from cfust_inputs import make_design, workload
    from cfust_inputs.synth import restart_params

    ds = workload("cfust_n1000_p2_q2_g2")
    qmc = cf.device_qmc(make_design(1024, 4, seed=1606), prec, device=dev)
    y = torch.as_tensor(ds.y_soa, device=dev)
    starts = restart_params(7, nstarts)
    n, p = ds.y.shape

    def make():
        return [(y, cf.device_params(P, device=dev), cf.alloc_estep(n, p, 2, 2, prec, device=dev, stderr=False))
                for P in starts]

    fb, fs = make(), make()
    B = cf.Batch(fb, qmc, handle=h)
    B.tune()
    B.fit(1, tol=0.0, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trace, _ = B.fit(iters, tol=0.0, use_graph=True)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / iters
    for (yy, P, es) in fs[:2]:
        cf.cfust_estep(yy, P.clone(), qmc, out=es)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        for (yy, P, es) in fs:
            cf.cfust_estep(yy, P, qmc, out=es)
            cf.cfust_mstep(yy, es, P, out=P)
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3 / iters
    B.close()
    pairs = nstarts * n * 2
    return {"fits": nstarts, "n": n, "p": p, "q": 2, "g": 2, "N": 1024, "S": 4,
            "batched_ms_per_iteration": ms_b, "sequential_ms_per_iteration": ms_s,
            "speedup": ms_s / ms_b, "batched_value": pairs / (ms_b / 1e3),
            "sequential_value": pairs / (ms_s / 1e3), "unit": "(obs*comp)/s"}


def batched_run(cf, h, prec, dev, steps: int, warmup: int, with_cpu: bool, precision_name: str,
                n_lo: float = 5e3, n_hi: float = 2e5, restarts: bool = True) -> dict:
    """The restart workload: 64 independent fits (n ~ logU[n_lo, n_hi], p = q
    in 3..8, g in 2..6) run as one batch, one step = one EM iteration of every
    fit (a replay of the captured graph), against the same fits run one after
    the other through the single-fit calls.  Both produce the same
    log-likelihoods bit for bit (checked), i.e. they are compared at equal
    accuracy."""
    import numpy as np
    import torch

    from cfust_inputs import make_design, workload

    progress(f"batched: drawing 64 fits, n ~ logU[{n_lo:g}, {n_hi:g}]")
    sets = workload("batched_fit", n_lo=n_lo, n_hi=n_hi)
    N, S = sets[0].meta["N"], sets[0].meta["S"]
    design = make_design(N, S, seed=1606)
    qmc = cf.device_qmc(design, prec, device=dev)

    def make():
        fits = []
        for ds in sets:
            n, p = ds.y.shape
            fits.append((torch.as_tensor(ds.y_soa, device=dev), cf.device_params(ds.params, device=dev),
                         cf.alloc_estep(n, p, ds.params.q, ds.params.g, prec, device=dev, stderr=False)))
        return fits

    fb, fs = make(), make()
    pairs = sum(int(ds.y.shape[0]) * ds.params.g for ds in sets)
    rows = sum(int(ds.y.shape[0]) for ds in sets)
    B = cf.Batch(fb, qmc, handle=h)
    progress("batched: tuning queues")
    tuned = B.tune()
    # batched: warm-up iterations, then the timed ones (graph replays)
    progress("batched: warm-up")
    B.fit(max(warmup, 1), tol=0.0, use_graph=True)
    torch.cuda.synchronize()
    for (_, dp, _), ds in zip(fb, sets):          # restart from the initial parameters
        src = cf.device_params(ds.params, device=dev)
        for f in ("pi", "mu", "Sigma", "Delta", "nu"):
            getattr(dp, f).copy_(getattr(src, f))
    torch.cuda.synchronize()
    progress("batched: timed")
    t0 = time.perf_counter()
    trace, done = B.fit(steps, tol=0.0, use_graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_batched = (t1 - t0) * 1e3 / steps

    # sequential: the same fits one after the other, same number of iterations
    for ds in {ds.params.q: ds for ds in sets}.values():
        h.autotune(torch.as_tensor(ds.y_soa[:, :4096].copy(), device=dev), cf.device_params(ds.params, device=dev),
                   qmc)
    progress("sequential: warm-up")
    for (y, P, es) in fs[:4]:
        cf.cfust_estep(y, P.clone(), qmc, out=es)
    torch.cuda.synchronize()
    progress("sequential: timed")
    seq_trace = torch.zeros((steps, len(fs)), dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    for it in range(steps):
        for k, (y, P, es) in enumerate(fs):
            cf.cfust_estep(y, P, qmc, out=es)
            seq_trace[it, k].copy_(es.loglik[0])
            cf.cfust_mstep(y, es, P, out=P)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_seq = (t1 - t0) * 1e3 / steps
    equal = bool(torch.equal(seq_trace, trace))

    # lattice kernel time of one batched E-step (events around the queue kernels)
    progress("batched: profiled E-step")
    h.profile(True)
    h.profile_read()
    B.estep()
    torch.cuda.synchronize()
    prof = h.profile_read()
    h.profile(False)
    points = {}
    for ds in sets:
        n = int(ds.y.shape[0])
        for m in integral_dims(ds.params.q):
            points[m] = points.get(m, 0) + N * S * n * ds.params.g
    roofline = lattice_roofline(prof, points, 1, "k_queue_grid / k_queue_qmc (lattice queue kernels in the "
                                                 "tuned form, one batched E-step)")
    out = {"value": pairs / (ms_batched / 1e3), "unit": "(obs*comp)/s", "steps": steps,
           "ms_per_step": ms_batched,
           "config": {"workload": "batched_fit", "n_range": [n_lo, n_hi], "fits": len(sets), "rows": rows,
                      "pairs": pairs,
                      "N": N, "S": S, "precision": precision_name,
                      "step": "one EM iteration of every fit (graph replay)",
                      "tuned_queues": {f"m{m}": {"rows": v[0], "blocks_per_slot": v[1], "points_per_lane": v[2]}
                                       for m, v in tuned.items()}},
           "roofline": roofline,
           "batched_vs_sequential": {"sequential_ms_per_step": ms_seq, "batched_ms_per_step": ms_batched,
                                     "speedup": ms_seq / ms_batched,
                                     "sequential_value": pairs / (ms_seq / 1e3),
                                     "loglik_traces_bit_equal": equal}}
    B.close()
    del fb, fs
    if restarts:
        progress("small restarts: 64 starts on the n = 1000 data")
        out["small_restarts"] = small_restarts(cf, h, prec, dev)
    if with_cpu:
        # one fit per q (the cost of a row depends on q and grows with g):
        # max(1, threads // g) rows of it, per-row time scaled by g to every
        # fit of that q and multiplied by its n
        import oracle
        oracle.build(force=False)
        threads = oracle.get_threads()
        per_row_comp, c_tot, sample_rows = {}, 0.0, 0
        for ds in sets:
            q, g = ds.params.q, ds.params.g
            if q in per_row_comp:
                continue
            r = max(1, threads // g)
            c0 = time.perf_counter()
            oracle.estep(ds.y, ds.params, design, rows=np.arange(r, dtype=np.int32))
            dt = time.perf_counter() - c0
            progress(f"cpu baseline: q = {q}, g = {g}, {r} rows: {dt:.1f} s")
            per_row_comp[q] = dt / (r * g)
            c_tot += dt
            sample_rows += r
        est_s = sum(per_row_comp[ds.params.q] * ds.params.g * ds.y.shape[0] for ds in sets)
        out["cpu_baseline"] = {"value": pairs / est_s, "unit": "(obs*comp)/s", "cores": threads, "kind": "oracle",
                               "sample": f"E-step of max(1, {threads}//g) observations of the first fit of each q "
                                         f"({sample_rows} rows, {c_tot:.1f} s), per (row, component) time "
                                         f"extrapolated to all pairs of the fits of that q; same lattice "
                                         f"(N={N}, S={S}), FP64",
                               "host": host_cpu()}
    return out


def batched_main(args) -> dict:
    """--workload batched_fit: the restart workload as the headline line."""
    import torch

    import paper_1606_02054_amd as cf

    prec = cf.CFUST_MIXED if args.precision == "mixed" else cf.CFUST_FP64
    dev = torch.device("cuda:0")
    h = cf.default_handle(0)
    r = batched_run(cf, h, prec, dev, args.steps, args.warmup, not args.no_cpu, args.precision)
    out = {"metric": METRIC, "value": r.pop("value"), "unit": r.pop("unit"), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if prec == cf.CFUST_MIXED else "f64",
           "data": "synthetic (drawn from the CFUST hierarchy, seeded)"}
    r.pop("steps")
    out.update(r)
    return out


def cytometry_iteration(cf, h, dev, n: int = 1_000_000) -> dict:
    """One EM iteration of the cytometry-shaped workload at full size: n = 10^6
    observations, p = q = 8, g = 5 (38 lattice integrals of dimensions 6, 7, 8
    per pair), lattice 8192 x 8, mixed precision; the lattice points per lane
    are tuned on the first 32768 observations (the choice depends on m, N, S
    and precision only)."""
    import torch
    from cfust_inputs import make_design, workload

    progress(f"cytometry: drawing n = {n}")
    ds = workload("cfust_n1e6_p8_q8_g5_box1024", n=n)
    p, q, g = ds.y.shape[1], ds.params.q, ds.params.g
    N, S = ds.meta["N"], ds.meta["S"]
    qmc = cf.device_qmc(make_design(N, S, seed=1606), cf.CFUST_MIXED, device=dev)
    y = torch.as_tensor(ds.y_soa, device=dev)
    P = cf.device_params(ds.params, device=dev)
    nxt = P.clone()
    tuned = h.autotune(y[:, :32768].contiguous(), P, qmc)
    es = cf.alloc_estep(n, p, q, g, cf.CFUST_MIXED, device=dev)
    h.reserve(n, p, q, g, qmc)
    torch.cuda.synchronize()
    progress("cytometry: timed EM iteration")
    h.profile(True)
    h.profile_read()
    t0 = time.perf_counter()
    cf.cfust_estep(y, P, qmc, out=es)
    cf.cfust_mstep(y, es, P, out=nxt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile_read()
    h.profile(False)
    ms = (t1 - t0) * 1e3
    progress(f"cytometry: EM iteration {ms / 1e3:.1f} s")
    points = {}
    for m in integral_dims(q):
        points[m] = points.get(m, 0) + N * S * n * g
    return {"value": n * g / (ms / 1e3), "unit": "(obs*comp)/s", "ms_per_step": ms,
            "config": {"workload": "cfust_n1e6_p8_q8_g5_box1024", "n": n, "p": p, "q": q, "g": g, "N": N, "S": S,
                       "precision": "mixed", "step": "E-step + M-step (one EM iteration)",
                       "autotuned_points_per_lane": {f"m{m}": v for m, v in tuned.items()}},
            "loglik": float(es.loglik.cpu()[0]),
            "roofline": lattice_roofline(prof, points, 1, "k_estep_qmc (FP32 lattice integrand)")}


def cpu_baseline(ds, design, g: int, N: int, S: int, rows_n: int = 0) -> dict:
    """The FP64 oracle on the host cores on a bounded sample of the workload
    (its first observations x all components, same lattice): with every
    thread (the reported rate), with one thread, and with g threads -- one per
    component, the scheme of the paper's Sec. 4 (its runs used a quad-core
    machine)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    rows_n = rows_n or max(2, threads // 2)

    def run(nthreads, nrows):
        oracle.set_threads(nthreads)
        c0 = time.perf_counter()
        oracle.estep(ds.y, ds.params, design, rows=np.arange(nrows, dtype=np.int32))
        return time.perf_counter() - c0

    progress(f"CPU oracle: {rows_n} rows on {threads} threads ...")
    t_all = run(threads, rows_n)
    progress(f"CPU oracle: {t_all:.1f} s; one row on 1 thread ...")
    t_one = run(1, 1)
    progress(f"CPU oracle: {t_one:.1f} s; one row on {g} threads ...")
    t_g = run(g, 1)
    progress(f"CPU oracle: {t_g:.1f} s")
    oracle.set_threads(threads)
    return {"value": rows_n * g / t_all, "unit": "(obs*comp)/s", "cores": threads, "kind": "oracle",
            "sample": f"E-step of the first {rows_n} observations x {g} components, same lattice (N={N}, S={S}), "
                      f"FP64, {t_all:.1f} s",
            "one_thread": {"value": g / t_one, "cores": 1, "sample": f"first observation x {g} components, "
                                                                    f"{t_one:.1f} s"},
            "paper_style_g_threads": {"value": g / t_g, "cores": g,
                                      "sample": f"first observation x {g} components, one thread per component "
                                                f"(the decomposition of the paper's Sec. 4), {t_g:.1f} s"},
            "host": host_cpu()}


SWEEP_N, SWEEP_S, SWEEP_ROWS = 4096, 8, 2048


def counter_sweep(cf, dev) -> None:
    """One mixed-precision E-step for q = 8, 5 and 2 (lattice integrals of every
    dimension m = 2..8) at SWEEP_ROWS observations and lattice SWEEP_N x
    SWEEP_S, for a counter run of the lattice kernels (each wave of
    k_estep_qmc evaluates SWEEP_N x SWEEP_S lattice points)."""
    import numpy as np
    import torch
    from cfust_inputs import draw_params, make_design, sample_hierarchy
    qmc = cf.device_qmc(make_design(SWEEP_N, SWEEP_S, seed=1606), cf.CFUST_MIXED, device=dev)
    for q in (8, 5, 2):
        rng = np.random.default_rng(700 + q)
        P = draw_params(rng, q, q, 3, sigma="wishart")
        y, _ = sample_hierarchy(rng, P, SWEEP_ROWS)
        es = cf.cfust_estep(torch.as_tensor(np.ascontiguousarray(y.T), device=dev), cf.device_params(P, device=dev),
                            qmc)
        torch.cuda.synchronize()
        progress(f"counter sweep: q = {q} done (loglik {float(es.loglik.cpu()[0]):.1f})")


def summarize_counters(dbs, points_per_wave: int) -> dict:
    """Per-dimension figures of the FP32 lattice kernel k_estep_qmc<m, FP32, 1
    point per lane> (with or without the coordinate table) from rocprofv3 databases (counter runs of the same
    command): FP32 flops per lattice point (2 FMA + MUL + ADD + TRANS per
    wave / points per wave), VALU instructions per point, wave64 VALU
    instructions per CU per cycle (GRBM_GUI_ACTIVE summed over the 8 XCDs),
    the share issued as pairs (SQ_ACTIVE_INST_VALU2 counts 4-cycle slots
    with two VALU issues) and the VALU busy share of the issue slots of the
    1024 SIMDs (SQ_ACTIVE_INST_VALU counts a transcendental twice)."""
    import re
    import sqlite3
    acc = {}
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, name, duration, counter_name, counter_value from pmc_events").fetchall()
        per = {}
        for did, name, dur, cn, cv in rows:
            mm = re.search(r"k_estep_qmc<(\d), true, 1(?:, (?:true|false))?>", name)
            if not mm:
                continue
            e = per.setdefault(did, {"m": int(mm.group(1)), "dur": dur})
            e[cn] = e.get(cn, 0.0) + cv
        for e in per.values():
            a = acc.setdefault(e["m"], {"n": 0, "dur": [0.0, 0]})
            a["n"] += 1
            for k, v in e.items():
                if k in ("m", "dur"):
                    continue
                c = a.setdefault(k, [0.0, 0])
                c[0] += v
                c[1] += 1
            a["dur"][0] += e["dur"]
            a["dur"][1] += 1
    # each counter (and the duration) averaged over the dispatches that report
    # it: counters that appear in several passes are not double-counted
    acc = {m: {k: (v[0] / v[1] if isinstance(v, list) else v) for k, v in a.items()} for m, a in acc.items()}
    out = {}
    for m, a in sorted(acc.items()):
        r = {}
        waves = a.get("SQ_WAVES")
        if waves:
            pts = waves * points_per_wave / 64.0      # a wave64 instruction evaluates 64 lattice points
            if all(k in a for k in ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
                                    "SQ_INSTS_VALU_TRANS_F32")):
                r["flops_per_point"] = (2 * a["SQ_INSTS_VALU_FMA_F32"] + a["SQ_INSTS_VALU_MUL_F32"]
                                        + a["SQ_INSTS_VALU_ADD_F32"] + a["SQ_INSTS_VALU_TRANS_F32"]) / pts
                r["trans_per_point"] = a["SQ_INSTS_VALU_TRANS_F32"] / pts
            if "SQ_INSTS_VALU" in a:
                r["valu_per_point"] = a["SQ_INSTS_VALU"] / pts
        if "SQ_INSTS_VALU" in a and "GRBM_GUI_ACTIVE" in a:
            cyc = a["GRBM_GUI_ACTIVE"] / 8.0
            r["valu_per_cu_cycle"] = a["SQ_INSTS_VALU"] / 256.0 / cyc
            r["clock_ghz"] = cyc / (a["dur"] * 1e-9) / 1e9
            if "SQ_ACTIVE_INST_VALU2" in a:
                r["dual_issue_frac"] = 2.0 * a["SQ_ACTIVE_INST_VALU2"] / a["SQ_INSTS_VALU"]
            if "SQ_ACTIVE_INST_VALU2" in a and "SQ_ACTIVE_INST_VALU" in a:
                # VALU busy: issue slots taken (a transcendental takes two, a
                # pair one) per SIMD over the kernel's 4-cycle slots
                r["valu_slot_busy"] = ((a["SQ_ACTIVE_INST_VALU"] - a["SQ_ACTIVE_INST_VALU2"]) / 1024.0) / (cyc / 4.0)
        r["dispatches"] = a["n"]
        out[m] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfust_n20000_p4_q4_g3")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample rows (0: one per thread)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-vs-lattice comparison")
    ap.add_argument("--no-components", action="store_true",
                    help="skip the M-step and network roofline figures")
    ap.add_argument("--components-only", action="store_true",
                    help="run only the M-step and network roofline figures (one JSON line)")
    ap.add_argument("--n", type=int, default=0, help="observations (0: the workload's own n)")
    ap.add_argument("--no-cytometry", action="store_true",
                    help="skip the full-size cytometry-shaped EM iteration (n = 10^6, p = q = 8, g = 5)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-fit batched iteration")
    ap.add_argument("--counter-sweep", action="store_true",
                    help="only one E-step per q = 8, 5, 2 (lattice kernels of m = 2..8) for a counter run")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DB",
                    help="print the per-m lattice-kernel figures of rocprofv3 databases of a --counter-sweep "
                         "run (no GPU needed)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        print(json.dumps({"kernel_digest": kernel_digest(),
                          "per_m": summarize_counters(args.summarize_counters, SWEEP_N * SWEEP_S)}, indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the bench runs on one GPU only (the kernels take one GPU's share of the data); "
                                   "--gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1606_02054_amd as cf
    from cfust_inputs import make_design, workload

    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.counter_sweep:
        cf.default_handle(0)
        counter_sweep(cf, torch.device("cuda:0"))
        return
    if args.workload == "batched_fit":
        print(json.dumps(batched_main(args)), flush=True)
        return
    if args.components_only:
        cf.default_handle(0)
        print(json.dumps({"components": component_rooflines(cf, torch.device("cuda:0"))}), flush=True)
        return

    ds = workload(args.workload, **({"n": args.n} if args.n else {}))
    n, p = ds.y.shape
    q, g = ds.params.q, ds.params.g
    N, S = ds.meta["N"], ds.meta["S"]
    design = make_design(N, S, seed=1606)
    prec = cf.CFUST_MIXED if args.precision == "mixed" else cf.CFUST_FP64

    dev = torch.device("cuda:0")
    h = cf.default_handle(0)
    y = torch.as_tensor(ds.y_soa, device=dev)
    qmc = cf.device_qmc(design, prec, device=dev)
    start = cf.device_params(ds.params, device=dev)
    params = [start.clone(), start.clone()]
    h.reserve(n, p, q, g, qmc)
    es = cf.alloc_estep(n, p, q, g, prec, device=dev)

    def step(k):
        cur, nxt = params[k % 2], params[(k + 1) % 2]
        cf.cfust_estep(y, cur, qmc, out=es)
        cf.cfust_mstep(y, es, cur, out=nxt)

    tuned = h.autotune(y, start, qmc)
    progress(f"autotuned {args.workload}")
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    h.profile(True)
    h.profile_read()          # drop anything recorded before
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile_read()
    h.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    progress(f"timed {args.steps} EM iterations: {ms_step:.2f} ms each")
    pairs = n * g
    value = pairs / (ms_step / 1e3)
    ll = float(es.loglik.cpu()[0])

    # roofline of the lattice kernels (FP32 VALU)
    points = {}
    for m in integral_dims(q):
        points[m] = points.get(m, 0) + N * S * pairs
    traffic = None
    if args.workload == "cfust_n20000_p4_q4_g3" and prec == cf.CFUST_MIXED and not args.n and counters_current():
        traffic = TRAFFIC_MIB
    roofline = lattice_roofline(prof, points, args.steps, "k_estep_qmc (FP32 lattice integrand)", traffic)

    out = {"metric": METRIC, "value": value, "unit": "(obs*comp)/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if prec == cf.CFUST_MIXED else "f64",
           "data": "synthetic (drawn from the CFUST hierarchy, seeded)",
           "config": {"workload": args.workload, "n": n, "p": p, "q": q, "g": g, "N": N, "S": S,
                      "precision": args.precision, "step": "E-step + M-step (one EM iteration)",
                      "autotuned_points_per_lane": {f"m{m}": v for m, v in tuned.items()},
                      "loglik_last": ll},
           "roofline": roofline}

    if not args.no_surrogate and prec == cf.CFUST_MIXED:
        out["surrogate"] = surrogate_vs_lattice(cf, ds, y, start, design, n * g)
        progress("surrogate section done")
    if not args.no_components and args.workload == "cfust_n20000_p4_q4_g3":
        out["component_rooflines"] = component_rooflines(cf, dev)
        progress("component rooflines done")
        out["initialisation"] = initialisation(cf, ds, y, qmc, dev)
        progress("initialisation done")
        out["precision_split"] = precision_split(cf, y, start, design, dev)
        out["small_fit"] = small_fit(cf, dev)
        progress("small fit done")

    default_run = args.workload == "cfust_n20000_p4_q4_g3" and prec == cf.CFUST_MIXED and not args.n
    if default_run and not args.no_cytometry:
        out["cytometry"] = cytometry_iteration(cf, h, dev)
        progress("cytometry section done")
    if default_run and not args.no_batched:
        out["batched"] = batched_run(cf, h, prec, dev, 1, 1, False, args.precision)
        out["batched"]["small_uneven_fits"] = batched_run(cf, h, prec, dev, 3, 1, False, args.precision,
                                                          n_lo=500, n_hi=5000, restarts=False)
        progress("batched section done")

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ds, design, g, N, S, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
