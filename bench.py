#!/usr/bin/env python3
"""Benchmark of the BBMM hot path on one MI355X.

Workload (N = 1,048,576 split into two independent models, as the paper trains
diagonal and off-diagonal pair energies separately): n = 917,504 and
n = 131,072 clustered MOB-ML-shaped feature rows, d = 48, Matern-5/2 ARD,
sigma^2 = 1e-3, block [y | 15 Rademacher probes], rank-100 pivoted-Cholesky
preconditioner, mBCG to relative residual 1e-6 (max 100 iterations).

A step is one BBMM training evaluation of both models (gp_mll_and_grad:
preconditioner, probes, mBCG with the fused K_hat V products, stochastic
Lanczos quadrature, gradient), BF16x3 products.  `value` is the nominal
K_hat V throughput over the whole step: sum of 2 n^2 (d + t) per product
divided by the step wall time, inputs resident in HBM.

Also reported: the tile-sweep kernel's own throughput from HIP events recorded
on its stream (the roofline entry), mBCG iterations/s, the same step in the
FP32 form and its agreement with the BF16x3 step, sampled-row error of the
product against the FP64 oracle, the oracle timed on host cores on a bounded
sample (cpu_baseline), and p50/p99 latency of a Poisson serving run (200 requests/s, 5 s warm-up, 60 s
measured) on the n = 262,144 serving model.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


SWEEP_COUNTERS = os.path.join(ROOT, "profiles", "sweep_bf16x3_n917504_t16_counters.md")


def _definition(text, name):
    """Source text of the first definition of `name` (function or struct template) in `text`: from the
    template/declaration line through its matching closing brace."""
    import re
    m = re.search(r"(?m)^(template <[^\n]*>\n)?[^\n]*\b" + re.escape(name) + r"\b[^;\n]*\{", text)
    if not m:
        return ""
    depth, i = 0, text.index("{", m.start())
    for j in range(i, len(text)):
        depth += {"{": 1, "}": -1}.get(text[j], 0)
        if depth == 0:
            return text[m.start():j + 1]
    return ""


# The sweep kernel and everything it executes: its source text decides whether recorded counters apply.
SWEEP_SOURCES = [("paper_2109_09817_amd/csrc/kmm.hip", ["profile_scaled", "NAOf", "ChunkUnits", "sweep_bf16x3_kernel"]),
                 ("paper_2109_09817_amd/csrc/mfma_bf16.h", ["f16_residual_pair", "split_f16x8", "mfma_val", "mfma_dist",
                                                            "vperm"])]


def sweep_source_digest():
    import hashlib
    h = hashlib.sha256()
    for path, names in SWEEP_SOURCES:
        with open(os.path.join(ROOT, path)) as fh:
            text = fh.read()
        for name in names:
            h.update(_definition(text, name).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per n = 917,504 sweep launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on a copy kernel), or None when the sweep's source has changed since."""
    try:
        text = open(SWEEP_COUNTERS).read()
    except OSError:
        return None
    vals = dict(l.split(" = ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_launch", "sweep_source_sha256")))
    if "sweep_source_sha256" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"]) if vals["sweep_source_sha256"].strip() == sweep_source_digest() else None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-form comparison step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-altbbmm", action="store_true", help="skip the AltBBMM solve")
    ap.add_argument("--no-protocol", action="store_true",
                    help="skip the AltBBMM protocol (exact GP on 50 molecules, then the FP64 full-set solve)")
    ap.add_argument("--serve-requests", type=int, default=12000,
                    help="measured window: this many Poisson arrivals at --serve-rate (12,000 at 200/s: about 60 s)")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="Poisson load before the measured window")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--profile-kmm", type=int, default=0, metavar="K",
                    help="profiling mode: a 1 GiB device copy (traffic calibration) then K products "
                         "K_hat V at n = 917,504, t = 16 (BF16x3), and exit")
    ap.add_argument("--profile-grad", type=int, default=0, metavar="K",
                    help="profiling mode: a 1 GiB device copy (traffic calibration) then K gradient sweeps "
                         "gp_kmm_grad at n = 917,504, t = 16 (BF16x3), and exit")
    ap.add_argument("--fit-c4", type=int, default=0, metavar="K",
                    help="training mode: K Adam steps (lr 0.05 on log theta, start l = 1, s_f = 1, "
                         "sigma^2 = 1e-2) on the n = 262,144, d = 48 model with t = 32 probes, and exit")
    ap.add_argument("--profile-exact", type=int, default=0, metavar="K",
                    help="profiling mode: K exact-GP evaluations (gp_exact_mll_and_grad) on the 50-molecule "
                         "subset of the n = 131,072 model, and exit")
    ap.add_argument("--profile-fp64", type=int, default=0, metavar="K",
                    help="profiling mode: K FP64 products K_hat V at n = 131,072 for t = 16 and t = 50, and exit")
    ap.add_argument("--noise-sweep", action="store_true",
                    help="low-noise mode: mBCG (pivoted Cholesky rank 100, [y | 15 probes], tol 1e-6) at "
                         "sigma^2 = 1e-2 .. 1e-8 with BF16x3, FP32 and FP64 products on two n = 16,384 "
                         "data sets, true residuals from FP64 products; product timings at n = 131,072; exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(row-sharding across GPUs is a design note, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2109_09817_amd import _lib, gp

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2109_09817_amd import build
        build.build()
    _lib.load()
    dev = torch.device("cuda:0")

    if args.profile_kmm:
        profile_kmm(args, gp, synth, torch, dev)
        return
    if args.profile_grad:
        profile_grad(args, gp, synth, torch, dev, np)
        return
    if args.fit_c4:
        fit_c4(args, synth, torch, dev, np)
        return
    if args.noise_sweep:
        noise_sweep(gp, _lib, synth, torch, dev, np)
        return
    if args.profile_exact:
        profile_exact(args, gp, synth, torch, dev, np)
        return
    if args.profile_fp64:
        profile_fp64(args, gp, synth, torch, dev)
        return

    names = [("c3o", 917504), ("c3d", 131072)]
    probs = {}
    for name, n in names:
        t0 = time.perf_counter()
        p = synth.make_problem(name)
        assert p.X.shape[0] == n
        probs[name] = dict(p=p, X=torch.from_numpy(p.X).to(dev), y=torch.from_numpy(p.y).to(dev),
                           k=gp.Kernel(p.ell, p.sf, p.noise))
        log(f"data {name}: n={n} d={p.X.shape[1]} ({time.perf_counter() - t0:.1f}s)")
    cfg = synth.CONFIGS["c3o"]
    t_cols = cfg.probes + 1

    def step(prec, seed):
        out = {}
        for name, _ in names:
            q = probs[name]
            r = gp.mll_and_grad(q["k"], q["X"], q["y"], probes=cfg.probes, rank=cfg.rank, max_iter=cfg.max_iter,
                                tol=cfg.tol, seed=seed, precision=prec)
            out[name] = r
        return out

    for w in range(args.warmup):
        step("bf16x3", 1000 + w)
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    gp.profile_read(reset=True)
    gp.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for s in range(args.steps):
        res.append(step("bf16x3", 2000 + s))
        log(f"step {s} done: " + ", ".join(f"{k} mll={v.mll:.6g} iters={v.info['iters']}" for k, v in res[-1].items()))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = gp.profile_records()
    launches, kms, kflops = gp.profile_read(reset=True)
    gp.profile_enable(False)
    # the dominant launch: the n = 917,504 square product of the 16-column block
    big = [r for r in recs if r[0] == 917504 and r[1] == 917504]
    big_ms = sum(r[3] for r in big) / len(big) if big else None
    big_flops = 2.0 * 917504 * 917504 * (48 + t_cols)
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = kflops / wall / 1e12
    kernel_tflops = big_flops / (big_ms * 1e-3) / 1e12 if big_ms else None
    iters = sum(r.info["iters"] for st in res for r in st.values())
    mbcg_ms = sum(r.info["ms_mbcg"] for st in res for r in st.values())
    phases = {k: sum(r.info[k] for st in res for r in st.values()) / args.steps
              for k in ("ms_precond", "ms_mbcg", "ms_grad")}

    extra = {
        "kmm_sweep_launches": launches,
        "kmm_sweep_ms_all_launches": kms,
        "kmm_sweep_tflops_all_launches": kflops / (kms * 1e-3) / 1e12 if kms > 0 else None,
        "kmm_sweep_n917504_launches": len(big),
        "kmm_sweep_n917504_ms_avg": big_ms,
        "mbcg_iters_per_s": iters / (mbcg_ms * 1e-3) if mbcg_ms > 0 else None,
        "mbcg_iters_per_step": {name: res[-1][name].info["iters"] for name, _ in names},
        "phase_ms_per_step": phases,
        "mll": {name: res[-1][name].mll for name, _ in names},
    }

    # the same step in the FP32 form, and its agreement with the BF16x3 step
    if not args.no_fp32:
        # the same warm-up and timed steps, with the same probe seeds, as the BF16x3 form
        for w in range(args.warmup):
            step("fp32", 1000 + w)
        torch.cuda.synchronize()
        gp.profile_read(reset=True)
        gp.profile_enable(True)
        t2 = time.perf_counter()
        res32 = []
        for s_ in range(args.steps):
            res32.append(step("fp32", 2000 + s_))
            log(f"fp32 step {s_} done")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        f32 = res32[-1]
        recs32 = gp.profile_records()
        _, kms32, kfl32 = gp.profile_read(reset=True)
        gp.profile_enable(False)
        big32 = [r for r in recs32 if r[0] == 917504 and r[1] == 917504]
        big32_ms = sum(r[3] for r in big32) / len(big32) if big32 else None
        mixed = res[-1]
        agree = {}
        for name, _ in names:
            a, b = mixed[name], f32[name]
            g_scale = max(np.abs(b.grad).max(), 1e-300)
            agree[name] = {
                "mll_rel": abs(a.mll - b.mll) / abs(b.mll),
                "quad_rel": abs(a.info["quad"] - b.info["quad"]) / abs(b.info["quad"]),
                "grad_max_rel": float(np.max(np.abs(a.grad - b.grad) / np.maximum(np.abs(b.grad), 1e-3 * g_scale))),
            }
        ph32 = {k: sum(r.info[k] for st in res32 for r in st.values()) / args.steps
                for k in ("ms_precond", "ms_mbcg", "ms_grad")}
        ms32 = (t3 - t2) * 1e3 / args.steps
        extra["fp32_form"] = {
            "ms_per_step": ms32,
            "phase_ms_per_step": ph32,
            "value_tflops": kfl32 / (t3 - t2) / 1e12,
            "kmm_sweep_tflops_nominal": kfl32 / (kms32 * 1e-3) / 1e12 if kms32 > 0 else None,
            "kmm_sweep_n917504_ms_avg": big32_ms,
            # the same K_hat V algorithm in both forms: the ratio of precision alone
            "kmm_sweep_speedup_bf16x3_over_fp32": big32_ms / big_ms if big32_ms and big_ms else None,
            "mbcg_phase_speedup_bf16x3_over_fp32": ph32["ms_mbcg"] / phases["ms_mbcg"],
            # the step ratio mixes precision and algorithm: the FP32 form's gradient runs the full-matrix
            # sweep (every ordered pair), the BF16x3 form's the upper triangle (each pair once)
            "step_speedup_bf16x3_over_fp32_mixed_algorithms": ms32 / ms_per_step,
            "timing": f"{args.warmup} untimed and {args.steps} timed FP32 steps after the BF16x3 steps, the same probe seeds",
            "agreement_bf16x3_vs_fp32": agree,
        }
        log(f"fp32 step: {ms32:.0f} ms")

    cpu = None
    if not args.no_cpu:
        cpu, extra["kmm_vs_oracle_sampled_rows"], extra["cpu_vs_gpu_ops"] = cpu_baseline_leg(
            gp, synth, torch, dev, np, probs["c3o"], t_cols)

    if not args.no_serve:
        extra["serving"] = serve_leg(args, gp, synth, torch, dev, np)
    if not args.no_altbbmm:
        extra["altbbmm"] = altbbmm_leg(gp, synth, torch, dev, np)
    if not args.no_protocol:
        extra["altbbmm_protocol"] = protocol_leg(gp, synth, torch, dev, np, probs["c3d"])

    out = {
        "metric": "K̂·V TFLOP/s + mBCG iters/s at N=1M (mixed vs FP32, rel err 1e-4); p99 predict latency",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16x3 distance and tile.V products (FP32 accumulate) / f64 solver",
        "data": "synthetic",
        "config": {"workload": "BBMM mll+gradient step, N=1,048,576 as two models (917,504 + 131,072 rows), "
                               "d=48, Matern-5/2 ARD, sigma^2=1e-3, [y | 15 probes], rank-100 pivoted Cholesky, "
                               "mBCG tol 1e-6", "n": [917504, 131072], "d": 48, "t": t_cols},
        "roofline": {"bound": "mfma", "achieved": kernel_tflops, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": kernel_tflops / PEAK_BF16_TFLOPS if kernel_tflops else None, "traffic": measured_traffic(),
                     "kernel": "sweep_bf16x3_kernel<5,1,MATERN52> at n=917,504, t=16",
                     "work": "2 n^2 (d + t) = 1.080e14 nominal flops per launch", "avg_launch_ms": big_ms},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def profile_kmm(args, gp, synth, torch, dev):
    """Kernels to read hardware counters on: one plain copy of known size, then K products."""
    p = synth.make_problem("c3o")
    X = torch.from_numpy(p.X).to(dev)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    V = torch.from_numpy(synth.random_block(p.X.shape[0], 16, 3)).to(dev)
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    out = torch.empty_like(V)
    gp.profile_enable(True)
    for _ in range(args.profile_kmm):
        gp.kmm(k, X, V, precision="bf16x3", out=out)
    torch.cuda.synchronize()
    recs = gp.profile_records()
    gp.profile_read(reset=True)
    print(json.dumps({"profile_kmm": {"copy_bytes": 2 * a.numel() * 8, "launch_ms": [r[3] for r in recs]}}),
          flush=True)


def profile_grad(args, gp, synth, torch, dev, np):
    """K hyperparameter-gradient sweeps on the n = 917,504 model, t = 16, to read counters on."""
    p = synth.make_problem("c3o")
    X = torch.from_numpy(p.X).to(dev)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    U = torch.from_numpy(synth.random_block(p.X.shape[0], 16, 4)).to(dev)
    W = torch.from_numpy(synth.random_block(p.X.shape[0], 16, 5)).to(dev)
    w = np.concatenate([[0.5], np.full(15, -0.5 / 15)])
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB: the traffic counters' calibration copy
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    ms = []
    for _ in range(args.profile_grad):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = gp.kmm_grad(k, X, U, W, w, precision="bf16x3")
        ms.append((time.perf_counter() - t0) * 1e3)
    print(json.dumps({"profile_grad": {"call_ms": ms, "grad0": float(g[0])}}), flush=True)


def profile_exact(args, gp, synth, torch, dev, np):
    """K exact-GP evaluations (mll, gradient) on the protocol's subset: 50 molecules of the n = 131,072 model."""
    p = synth.make_problem("c3d")
    sub = synth.molecule_subset(p.mol, 50, p.cfg.seed)
    X = torch.from_numpy(np.ascontiguousarray(p.X[sub])).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(p.y[sub])).to(dev)
    k = gp.Kernel(np.ones(p.X.shape[1]), 1.0, 1e-2)
    ms = []
    for _ in range(args.profile_exact):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gp.exact_mll_and_grad(k, X, y)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    print(json.dumps({"profile_exact": {"n": int(X.shape[0]), "call_ms": ms, "mll": r.mll}}), flush=True)


def profile_fp64(args, gp, synth, torch, dev):
    """K FP64 products on the n = 131,072 model at t = 16 (mBCG block) and t = 50 (block CG block)."""
    p = synth.make_problem("c3d")
    X = torch.from_numpy(p.X).to(dev)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    n = p.X.shape[0]
    out = {}
    for t in (16, 50):
        V = torch.from_numpy(synth.random_block(n, t, 3)).to(dev)
        W = torch.empty_like(V)
        ms = []
        for _ in range(args.profile_fp64):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gp.kmm(k, X, V, precision="fp64", out=W)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        out[f"t{t}_call_ms"] = ms
    print(json.dumps({"profile_fp64": out}), flush=True)


def fit_c4(args, synth, torch, dev, np):
    """Hyperparameter training on the gradient configuration: Adam on log theta through autograd.MLL."""
    from paper_2109_09817_amd import autograd as ag
    p = synth.make_problem("c4")
    X = torch.from_numpy(p.X).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    d = p.X.shape[1]
    start = np.concatenate([np.zeros(d), [0.0, math.log(1e-2)]])
    cfg = synth.CONFIGS["c4"]

    def progress(s, r):
        log(f"step {s}: mll {r.mll[-1]:.6e} iters {r.iters[-1]} {r.seconds[-1]:.3f} s")

    res = ag.fit(X, y, start, steps=args.fit_c4, lr=0.05, probes=cfg.probes, rank=cfg.rank,
                 max_iter=cfg.max_iter, tol=cfg.tol, seed=cfg.seed, callback=progress)
    th = np.exp(res.log_theta)
    print(json.dumps({"fit_c4": {
        "n": int(p.X.shape[0]), "d": d, "probes": cfg.probes, "steps": args.fit_c4,
        "s_per_step": float(np.mean(res.seconds[1:] if len(res.seconds) > 1 else res.seconds)),
        "first_step_s": res.seconds[0], "mll": res.mll, "mbcg_iters": res.iters,
        "final": {"lengthscale_min": float(th[:d].min()), "lengthscale_max": float(th[:d].max()),
                  "outputscale": float(th[d]), "noise": float(th[d + 1])}}}), flush=True)


def noise_sweep(gp, _lib, synth, torch, dev, np):
    """Where each product precision stops resolving K_hat (Sec. 3.2: rounding beyond the noise breaks
    the solver), and AltBBMM (FP64 block CG, Nystrom rank 1024) beside mBCG.  Two n = 16,384 data sets:
    the ill-conditioned variant of the n = 65,536 workload's layout, and the same layout with nearly
    repeated pairs of rows (lambda_min(K) ~ 1e-5)."""
    n, t, rank, tol, max_iter = 16384, 15, 100, 1e-6, 1500
    out = {"n": n, "probes": t, "rank": rank, "tol": tol, "max_iter": max_iter, "runs": []}
    p = synth.make_problem("c2", n=n, cond_variant=True)
    sets = [("ill_conditioned", p.X, p.y, p.ell), ("near_duplicate_pairs",) + synth.near_duplicate_pairs(n, 7)]
    for label, Xh, yh, ell in sets:
        X = torch.from_numpy(Xh).to(dev)
        y = torch.from_numpy(yh).to(dev)
        for noise in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
            k = gp.Kernel(ell, 1.0, noise)
            pc = gp.pivchol(k, X, rank)
            B = gp.probe_block(y, t, 5, noise, pc)
            for prec in ("bf16x3", "fp32", "fp64"):
                rec = {"data": label, "noise": noise, "precision": prec}
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                try:
                    r = gp.mbcg(k, X, B, max_iter, tol, pc=pc, precision=prec, want_z0=False)
                except _lib.GpError as e:
                    rec.update(status="breakdown", error=str(e), seconds=time.perf_counter() - t0)
                    out["runs"].append(rec)
                    log(f"noise {label} {noise:.0e} {prec}: breakdown ({e})")
                    continue
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                KU = gp.kmm(k, X, r.U[:1].contiguous(), precision="fp64")
                true = float(torch.linalg.norm(KU[0] - y) / torch.linalg.norm(y))
                rec.update(status="converged" if r.status == 0 else "max_iter", iters=int(r.iters.max()),
                           y_iters=int(r.iters[0]), relres_max=float(r.relres.max()), true_relres_y=true,
                           seconds=dt, ms_per_iter=dt / max(1, int(r.iters.max())) * 1e3)
                out["runs"].append(rec)
                log(f"noise {label} {noise:.0e} {prec}: {rec['status']} {rec['iters']} it, y: recurrence "
                    f"{r.relres[0]:.1e} true {true:.1e}, {dt:.2f} s")
            # AltBBMM: FP64 block CG on [y | 15 probes] with the rank-1024 Nystrom preconditioner
            rec = {"data": label, "noise": noise, "precision": "fp64", "solver": "altbbmm"}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                M = np.sort(np.random.default_rng(np.random.SeedSequence([17, 12])).choice(n, 1024, replace=False))
                ny = gp.nystrom_precond(k, X, M)
                Bb = torch.cat([y[None, :], torch.from_numpy(synth.random_block(n, t, 11)).to(dev)])
                r = gp.bcg(k, X, Bb, max_iter, tol, pc=ny, precision="fp64")
            except _lib.GpError as e:
                rec.update(status="breakdown", error=str(e), seconds=time.perf_counter() - t0)
                out["runs"].append(rec)
                log(f"noise {label} {noise:.0e} altbbmm fp64: breakdown ({e})")
            else:
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                KU = gp.kmm(k, X, r.W[:1].contiguous(), precision="fp64")
                true = float(torch.linalg.norm(KU[0] - y) / torch.linalg.norm(y))
                rec.update(status="converged" if r.status == 0 else "max_iter", iters=int(r.iters),
                           relres_max=float(r.relres.max()), true_relres_y=true, seconds=dt, kept=ny.kept)
                out["runs"].append(rec)
                log(f"noise {label} {noise:.0e} altbbmm fp64: {rec['status']} {r.iters} it, y true {true:.1e}, "
                    f"{dt:.2f} s (Nystrom kept {ny.kept})")
                del ny, Bb, r
            del pc, B
        del X, y
        torch.cuda.empty_cache()
    # the three product forms at n = 131,072, t = 16
    p = synth.make_problem("c3d")
    X = torch.from_numpy(p.X).to(dev)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    V = torch.from_numpy(synth.random_block(p.X.shape[0], 16, 3)).to(dev)
    W = torch.empty_like(V)
    nn = p.X.shape[0]
    out["products_n131072_t16"] = {}
    for prec in ("bf16x3", "fp32", "fp64"):
        gp.kmm(k, X, V, precision=prec, out=W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            gp.kmm(k, X, V, precision=prec, out=W)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        out["products_n131072_t16"][prec] = {"ms": ms,
                                             "tflops_nominal": 2.0 * nn * nn * (p.X.shape[1] + 16) / ms / 1e9}
        log(f"product n={nn} t=16 {prec}: {ms:.2f} ms")
    print(json.dumps({"noise_sweep": out}), flush=True)


def altbbmm_leg(gp, synth, torch, dev, np):
    """AltBBMM solves (Sec. 3.2): block CG, s = 50 ([y | 49 N(0, 1) columns]), tolerance 1e-6 on every
    column, with the symmetric Nystrom preconditioner of rank 512 over random landmark rows and without
    it: the n = 131,072 and n = 917,504 models as configured (nearly diagonal kernels), and the
    ill-conditioned variant (lengthscales x sqrt(2d)) at n = 16,384 with FP32 products."""
    out = {"s": 50, "rank": 512, "tol": 1e-6}
    cases = [("c3d", "c3d", None, False, "bf16x3"), ("c3o", "c3o", None, False, "bf16x3"),
             ("c2_ill_conditioned_n16384", "c2", 16384, True, "fp32")]
    for label, name, nsub, cond, prec in cases:
        p = synth.make_problem(name, n=nsub, cond_variant=cond) if nsub else synth.make_problem(name)
        n = p.X.shape[0]
        X = torch.from_numpy(p.X).to(dev)
        k = gp.Kernel(p.ell, p.sf, p.noise)
        B = np.vstack([p.y[None, :], synth.random_block(n, 49, 11)])
        Bd = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
        M = np.sort(np.random.default_rng(np.random.SeedSequence([p.cfg.seed, 12])).choice(n, 512, replace=False))
        rec = {"n": n, "precision": prec}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = gp.nystrom_precond(k, X, M)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = gp.bcg(k, X, Bd, 200, 1e-6, pc=pc, precision=prec)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plain = gp.bcg(k, X, Bd, 200, 1e-6, pc=None, precision=prec)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        flops = res.iters * 2.0 * n * n * (p.X.shape[1] + 50)
        rec["nystrom"] = {"precond_s": t1 - t0, "solve_s": t2 - t1, "iters": res.iters,
                          "relres_max": float(res.relres.max()), "status": res.status,
                          "products_tflops_nominal": flops / (t2 - t1) / 1e12}
        rec["unpreconditioned"] = {"solve_s": t3 - t2, "iters": plain.iters, "relres_max": float(plain.relres.max()),
                                   "status": plain.status}
        log(f"altbbmm {label}: Nystrom precond {t1 - t0:.2f} s + solve {t2 - t1:.2f} s ({res.iters} it); "
            f"unpreconditioned {t3 - t2:.2f} s ({plain.iters} it)")
        out[label] = rec
        del pc, res, plain, Bd, X
        torch.cuda.empty_cache()
    out["paper_rank"] = altbbmm_paper_rank(gp, synth, torch, dev, np)
    return out


def altbbmm_paper_rank(gp, synth, torch, dev, np, r=10000):
    """AltBBMM at the paper's preconditioner rank (Sec. 4: r = 10^4, s = 50, tol 1e-6) on the n = 131,072
    model: the Cholesky-factor Nystrom preconditioner (FP64 matrix-core products, no eigendecomposition)
    and block preconditioned CG with FP64 products (the paper's precision) and with BF16x3 products; then
    the ill-conditioned variant of the n = 65,536 layout with FP64 products, against no preconditioner."""
    p = synth.make_problem("c3d")
    n = p.X.shape[0]
    X = torch.from_numpy(p.X).to(dev)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    B = np.vstack([p.y[None, :], synth.random_block(n, 49, 11)])
    Bd = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    M = np.sort(np.random.default_rng(np.random.SeedSequence([p.cfg.seed, 13])).choice(n, r, replace=False))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc = gp.nystrom_chol_precond(k, X, M)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = p.X.shape[1]
    build_flops = 2.0 * 2 * n * r * r + 1.0 * n * r * r  # two n x r x r products and the Gram's lower tiles
    rec = {"n": n, "rank": r, "s": 50, "tol": 1e-6, "build_s": t1 - t0,
           "build_fp64_tflops_nominal": build_flops / (t1 - t0) / 1e12}
    log(f"altbbmm rank {r}: Cholesky-factor Nystrom build {t1 - t0:.2f} s")
    for prec in ("fp64", "bf16x3"):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        res = gp.bpcg(k, X, Bd, 200, 1e-6, pc=pc, precision=prec)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        plain = gp.bpcg(k, X, Bd, 200, 1e-6, pc=None, precision=prec)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        KW = gp.kmm(k, X, res.W[:1].contiguous(), precision="fp64")
        true = float(torch.linalg.norm(KW[0] - Bd[0]) / torch.linalg.norm(Bd[0]))
        rec[prec] = {"solve_s": tb - ta, "iters": res.iters, "status": res.status,
                     "relres_max": float(res.relres.max()), "true_relres_y": true,
                     "unpreconditioned": {"solve_s": tc - tb, "iters": plain.iters, "status": plain.status}}
        log(f"altbbmm rank {r} {prec}: {res.iters} it in {tb - ta:.2f} s (true residual {true:.1e}); "
            f"unpreconditioned {plain.iters} it in {tc - tb:.2f} s")
        del res, plain, KW
    del pc, Bd, X
    torch.cuda.empty_cache()
    # where the preconditioner pays: the ill-conditioned variant (lengthscales x sqrt(2d)) at n = 65,536
    q = synth.make_problem("c2", cond_variant=True)
    nq = q.X.shape[0]
    Xq = torch.from_numpy(q.X).to(dev)
    kq = gp.Kernel(q.ell, q.sf, q.noise)
    Bq = torch.from_numpy(np.ascontiguousarray(np.vstack([q.y[None, :], synth.random_block(nq, 49, 11)]))).to(dev)
    Mq = np.sort(np.random.default_rng(np.random.SeedSequence([q.cfg.seed, 13])).choice(nq, r, replace=False))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pcq = gp.nystrom_chol_precond(kq, Xq, Mq)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = gp.bpcg(kq, Xq, Bq, 1000, 1e-6, pc=pcq, precision="fp64")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plain = gp.bpcg(kq, Xq, Bq, 1000, 1e-6, pc=None, precision="fp64")
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    KW = gp.kmm(kq, Xq, res.W[:1].contiguous(), precision="fp64")
    true = float(torch.linalg.norm(KW[0] - Bq[0]) / torch.linalg.norm(Bq[0]))
    rec["c2_ill_conditioned_n65536_fp64"] = {
        "n": nq, "build_s": t1 - t0, "solve_s": t2 - t1, "iters": res.iters, "status": res.status,
        "true_relres_y": true, "unpreconditioned": {"solve_s": t3 - t2, "iters": plain.iters, "status": plain.status}}
    log(f"altbbmm rank {r}, ill-conditioned n={nq} fp64: build {t1 - t0:.2f} s, {res.iters} it in {t2 - t1:.2f} s "
        f"(true residual {true:.1e}); unpreconditioned {plain.iters} it in {t3 - t2:.2f} s")
    del pcq, res, plain, KW, Xq, Bq
    torch.cuda.empty_cache()
    return rec


def cpu_baseline_leg(gp, synth, torch, dev, np, q, t_cols):
    """The FP64 oracle timed on the host cores beside the GPU (the only place the benchmark runs it):
    its K_hat V on 512 sampled rows of the n = 917,504 model (the reported baseline, and the GPU
    products' error on those rows), then two whole operations at n = 2,048 (the n = 2,048, d = 32
    workload): the exact (dense Cholesky) mll and gradient, and one BBMM estimate (rank-20 pivoted
    Cholesky, 8 probes, 30 iterations), each against the library's."""
    from oracle import bbmm as obbmm, exact as oexact, kernel as ok
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = None
    p = q["p"]
    th = ok.Theta(p.ell, p.sf, p.noise)
    n = p.X.shape[0]
    V = synth.random_block(n, t_cols, 3)
    R = 512
    rows = np.random.default_rng(1).choice(n, R, replace=False)
    t0 = time.perf_counter()
    ref = ok.khat_matmul(p.X, th, V.T, rows=rows, block=128).T
    t1 = time.perf_counter()
    fl = 2.0 * R * n * (p.X.shape[1] + t_cols)
    cpu = {"value": fl / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": blas or 1, "kind": "oracle",
           "sample": f"FP64 oracle K_hat V for {R} sampled rows of the n=917,504 model (t={t_cols}); "
                     f"{t1 - t0:.1f} s; the oracle's product runs on {blas} BLAS threads of "
                     f"{os.cpu_count()} host cores, its distances (scipy cdist) on one of them"}
    log(f"cpu baseline: {cpu['value']:.3e} TFLOP/s in {t1 - t0:.1f}s")
    Vg = torch.from_numpy(V).to(dev)
    diag = (th.sf + th.noise) * V[:, rows]
    acc = {}
    for prec in ("bf16x3", "fp32"):
        W = gp.kmm(q["k"], q["X"], Vg, precision=prec)
        torch.cuda.synchronize()
        got = W.cpu().numpy()[:, rows]
        acc[prec] = {
            "rel_err": float(np.max(np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1))),
            "rel_err_offdiag": float(np.max(np.linalg.norm((got - diag) - (ref - diag), axis=1)
                                            / np.linalg.norm(ref - diag, axis=1))),
        }
        del W
    ops = []
    c1 = synth.make_problem("c1")
    th1 = ok.Theta(c1.ell, c1.sf, c1.noise)
    k1 = gp.Kernel(c1.ell, c1.sf, c1.noise)
    X1 = torch.from_numpy(c1.X).to(dev)
    y1 = torch.from_numpy(c1.y).to(dev)
    n1 = c1.X.shape[0]

    def gpu_time(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - ta) / reps, out

    t0 = time.perf_counter()
    g_ref = oexact.mll_grad(c1.X, c1.y, th1)
    m_ref = oexact.cholesky_gp(c1.X, c1.y, th1)["mll"]
    t1 = time.perf_counter()
    tg, r = gpu_time(lambda: gp.exact_mll_and_grad(k1, X1, y1))
    ops.append({"op": "exact mll + gradient (dense Cholesky)", "n": n1, "d": int(c1.X.shape[1]),
                "cpu_s": t1 - t0, "gpu_s": tg, "gpu_over_cpu_speed": (t1 - t0) / tg,
                "mll_rel_diff": abs(r.mll - m_ref) / abs(m_ref),
                "grad_max_abs_diff": float(np.max(np.abs(r.grad - g_ref)))})
    cfg = synth.CONFIGS["c1"]
    t0 = time.perf_counter()
    piv = [int(v) for v in gp.pivchol(k1, X1, cfg.rank).pivots]
    o = obbmm.mll_and_grad_estimate(c1.X, c1.y, th1, t=cfg.probes, k=cfg.rank, seed=3, max_iter=cfg.max_iter,
                                    tol=1e-12, pivots=piv)
    t1 = time.perf_counter()
    tg, r = gpu_time(lambda: gp.mll_and_grad(k1, X1, y1, probes=cfg.probes, rank=cfg.rank,
                                             max_iter=cfg.max_iter, tol=0.0, seed=3, precision="bf16x3"))
    ops.append({"op": "BBMM mll + gradient estimate (pivoted Cholesky, probes, mBCG, SLQ, gradient)", "n": n1,
                "probes": cfg.probes, "rank": cfg.rank, "iterations": cfg.max_iter, "cpu_s": t1 - t0, "gpu_s": tg,
                "gpu_over_cpu_speed": (t1 - t0) / tg, "mll_rel_diff": abs(r.mll - o["mll"]) / abs(o["mll"])})
    for op in ops:
        op["cores"] = blas or 1
        log(f"cpu vs gpu: {op['op']} n={op['n']}: cpu {op['cpu_s']:.2f} s, gpu {op['gpu_s'] * 1e3:.2f} ms")
    return cpu, acc, ops


def protocol_leg(gp, synth, torch, dev, np, q, steps=30):
    """The AltBBMM training protocol (Sec. 3.2, Sec. 4) on the n = 131,072 model: hyperparameters from the
    exact GP on 50 random molecules (Adam, lr 0.05, start l = 1, s_f = 1, sigma^2 = 1e-2), sigma^2_add = 1e-5,
    then block CG (s = 50, tol 1e-6) with FP64 products and the rank-512 Nystrom preconditioner."""
    from paper_2109_09817_amd import protocol
    p = q["p"]
    n, d = p.X.shape
    sub = synth.molecule_subset(p.mol, 50, p.cfg.seed)
    M = np.sort(np.random.default_rng(np.random.SeedSequence([p.cfg.seed, 12])).choice(n, 512, replace=False))
    Bx = synth.random_block(n, 49, 11)
    start = np.concatenate([np.zeros(d), [0.0, math.log(1e-2)]])

    def progress(s, r):
        if s % 10 == 0 or s == steps - 1:
            log(f"protocol subset step {s}: exact mll {r.mll[-1]:.6e} ({r.seconds[-1] * 1e3:.0f} ms)")

    res = protocol.altbbmm_train(q["X"], q["y"], sub, start, M, Bx, steps=steps, lr=0.05, noise_add=1e-5,
                                 tol=1e-6, max_iter=500, precision="fp64", callback=progress)
    KW = gp.kmm(res.kernel, q["X"], res.W[:1].contiguous(), precision="fp64")
    true = float(torch.linalg.norm(KW[0] - q["y"]) / torch.linalg.norm(q["y"]))
    ns = int(sub.size)
    step_s = float(np.median(res.fit.seconds[1:])) if steps > 1 else res.fit.seconds[0]
    th = np.exp(res.log_theta)
    out = {"n": n, "subset_molecules": 50, "subset_rows": ns, "adam_steps": steps,
           "exact_step_ms": step_s * 1e3,
           "exact_step_fp64_tflops_nominal": float(ns) ** 3 / step_s / 1e12,
           "exact_mll_first_last": [res.fit.mll[0], res.fit.mll[-1]],
           "hyperparameters": {"lengthscale_min": float(th[:d].min()), "lengthscale_max": float(th[:d].max()),
                               "lengthscale_mean_abs_log_err_vs_generating":
                                   float(np.mean(np.abs(res.log_theta[:d] - np.log(p.ell)))),
                               "outputscale": float(th[d]), "noise_opt": float(th[d + 1]),
                               "noise_full_set": res.kernel.noise},
           "solve": {"precision": "fp64", "s": 50, "rank": 512, "kept": res.kept, "iters": res.iters,
                     "status": res.status, "relres_max": float(res.relres.max()), "true_relres_y": true},
           "seconds": res.seconds}
    log(f"protocol: subset {ns} rows, exact step {step_s * 1e3:.0f} ms, mll {res.fit.mll[0]:.4e} -> "
        f"{res.fit.mll[-1]:.4e}; full solve {res.iters} it in {res.seconds['solve']:.2f} s (precond "
        f"{res.seconds['precond']:.2f} s), true residual {true:.1e}")
    return out


def serve_leg(args, gp, synth, torch, dev, np):
    """Poisson requests against the resident n = 262,144 serving model (the generating hyperparameters;
    alpha from mBCG to 1e-6 and a rank-256 Lanczos variance cache, both BF16x3 products): a warm-up
    window of Poisson load whose results are discarded, then the measured window."""
    from paper_2109_09817_amd.serve import GpuExecutor, Server, latency_summary
    t0 = time.perf_counter()
    p = synth.make_problem("c5")
    k = gp.Kernel(p.ell, p.sf, p.noise)
    X = torch.from_numpy(p.X).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    pc = gp.pivchol(k, X, 100)
    sol = gp.mbcg(k, X, y[None, :].contiguous(), max_iter=100, tol=1e-6, pc=pc, want_z0=False)
    if sol.status != 0 or not float(sol.relres[0]) <= 1e-6:
        raise RuntimeError(f"serving model: the alpha solve did not converge (status {sol.status}, "
                           f"relative residual {float(sol.relres[0]):.2e})")
    alpha = sol.U[0].contiguous()
    t1 = time.perf_counter()
    R, kc = gp.lanczos_cache(k, X, y, 256)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    model = gp.PredictModel(k, X, alpha, R)
    ex = GpuExecutor(model, slots=4, max_rows=2048)
    srv = Server(ex, d=p.X.shape[1], hbm_budget=2 << 30)

    def drive(duration, seed, count=None):
        reqs = synth.request_stream(args.serve_rate, duration, seed=seed, count=count)
        payload = [synth.query_molecule("c5", m, seed=s) for (_, m, s) in reqs]
        futs = []
        start = time.perf_counter()
        for (ta, m, s), Z in zip(reqs, payload):
            now = time.perf_counter() - start
            if ta > now:
                time.sleep(ta - now)
            futs.append(srv.submit(Z))
        results = [f.result() for f in futs]
        return results, time.perf_counter() - start

    warm, _ = drive(args.serve_warmup, seed=4) if args.serve_warmup > 0 else ([], 0.0)
    log(f"serving warm-up: {len(warm)} requests over {args.serve_warmup:.0f} s")
    results, wall = drive(None, seed=5, count=args.serve_requests)
    srv.close()
    summ = latency_summary(results, wall)
    summ.update({"model_n": p.X.shape[0], "model": "generating hyperparameters of the n = 262,144 serving model",
                 "cache_rank": kc, "cache_precision": "bf16x3", "rate_req_s": args.serve_rate,
                 "seconds": wall, "warmup_seconds": args.serve_warmup, "warmup_requests": len(warm),
                 "slots": 4, "hbm_budget_bytes": 2 << 30, "alpha_solve_iters": int(sol.alpha.shape[0]),
                 "alpha_relres": float(sol.relres[0]), "setup_s": {"alpha": t1 - t0, "lanczos_cache": t2 - t1}})
    log(f"serving: p50 {summ['p50_ms']:.2f} ms p99 {summ['p99_ms']:.2f} ms, {summ['requests']} requests")
    return summ


if __name__ == "__main__":
    main()
