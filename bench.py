#!/usr/bin/env python3
"""Throughput of the SegSALSA-STR SALSA loop on one MI355X.

Headline workload: the 2048 x 2048, K = 16, 5x5-patch, 500-round solve (the
largest single-GPU configuration).  One step = one call of segsalsa_str_solve
on it: initialisation and all 500 rounds (proximity operators, multiplier
updates, J^T scatter, FFT z-solve), inputs resident in device memory.  The
metric is pixel*class*rounds per second of the FP32 path; it counts only if
the FP32 z is within 2e-4 (max-abs) of the FP64 z of the same input after
the whole solve (the FP64 path is pinned to the FP64 CPU oracle by the GPU
tests).  The 64-image batch is reported as a second, named entry.  Printed
as one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel·class·iterations/sec of SALSA-STR loop, FP32 vs FP64 at z err ≤2e-4"
UNIT = "pixel·class·iterations/s"
HBM_PEAK_GBS = 8000.0
Z_TOL = 2e-4
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_1504_07028_amd/csrc/prox_kernel.hip", "paper_1504_07028_amd/csrc/prox_math.h",
                  "paper_1504_07028_amd/csrc/segsalsa_internal.h", "paper_1504_07028_amd/csrc/segsalsa_kernels.h",
                  "paper_1504_07028_amd/csrc/api.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def prox_bytes_per_unit(L: int, b: int) -> int:
    """Algorithmic bytes of the fused prox kernel per pixel*class: d2 read+write (4L words),
    d1/d3/d4 read+write (6), p_hat read (1), z read (1), right-hand side write (1)."""
    return (4 * L + 9) * b


def load_traffic(workload: str, dtype: str, src_hash: str):
    """Measured HBM bytes per prox launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(PROFILE_DIR, f"prox_{workload}_{dtype}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != src_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


def time_calls(torch, call, steps, warmup):
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


def phase_times(S, torch, call, steps):
    """Average per-launch GPU time of each phase, from HIP events recorded around every launch."""
    S.segsalsa_profile_read(reset=True)
    S.segsalsa_profile_enable(True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    S.segsalsa_profile_enable(False)
    tot = S.segsalsa_profile_read(reset=True)
    return {name: dict(avg_us=1e3 * tot[name][0] / max(1, tot[name][1]), launches=tot[name][1])
            for name in S.PHASES[:4]}


def cpu_baseline(wl, probs, weights, budget_s: float, crop: int = 256):
    """The FP64 oracle timed on this host on a bounded sample of the workload: the top-left
    crop x crop pixels of the same input (all K classes, same patch and parameters, periodic
    boundary on the crop), as many rounds as fit in about budget_s seconds.  The per-unit rate
    (pixel*class*rounds/s) is what is compared; the oracle's cost per unit does not depend on
    the image size except through the FFT's log factor."""
    from threadpoolctl import threadpool_limits
    from oracle import segsalsa_ref as R
    H, W = min(crop, wl.H), min(crop, wl.W)
    x = np.ascontiguousarray(probs[:, :H, :W])
    pr = R.Problem(np.asarray(weights, dtype=np.float64), wl.M, wl.schatten_p, wl.lam, wl.mu)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        R.solve(x, pr, 1)
        t1 = time.perf_counter() - t0
        rounds = int(max(1, min(wl.iters, budget_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        R.solve(x, pr, rounds)
        dt = time.perf_counter() - t0
    units = H * W * wl.K * rounds
    return dict(value=units / dt, unit=UNIT, cores=1, kind="oracle",
                sample=f"{wl.name}: its top-left {H}x{W} crop (K = {wl.K}, {2 * wl.M + 1}x{2 * wl.M + 1} patch), "
                       f"{rounds} rounds from the initial state, FP64 numpy, 1 thread (BLAS/FFT limited to 1), "
                       f"{dt:.1f} s; host reports {os.cpu_count()} logical CPUs")


def bench_adjoint(S, torch, synth, steps, warmup, ck=0):
    """Differentiable solve on the 256x256, K = 8, 3x3-patch, 50-round workload: one step is the
    checkpointed forward plus the reverse sweep (gradients w.r.t. logits, lambda, patch weights)
    of the cross-entropy of z against the label map.  ck = 0: the library's checkpoint interval."""
    wl = synth.WORKLOADS["diff_256x256_k8"]
    d = synth.make_workload(wl)
    units = wl.n * wl.K * wl.iters
    lab = torch.from_numpy(d["labels"]).long().cuda()
    out = {"workload": wl.name, "checkpoint_every": ck, "unit": "pixel·class·iterations/s (forward + backward)"}
    for dtype, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
        x = torch.from_numpy(d["logits"]).to(device="cuda", dtype=dtype)
        pr = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], wl.schatten_p, wl.lam, wl.mu, wl.iters,
                       input_is_logits=True)
        out["checkpoint_interval_" + tag] = S.segsalsa_str_grad_checkpoint_interval(pr, S._prec(dtype), ck)
        ws = torch.empty(S.segsalsa_str_grad_workspace_size(pr, S._prec(dtype), ck), dtype=torch.uint8,
                         device="cuda")
        z = torch.empty_like(x)
        S.segsalsa_str_solve_ckpt(pr, ck, x, z, ws)
        zd = z.double().requires_grad_(True)
        loss = -torch.log(torch.gather(zd, 0, lab[None])[0].clamp_min(1e-6)).mean()
        (gz,) = torch.autograd.grad(loss, zd)
        gz = gz.to(dtype).contiguous()
        gi = torch.empty_like(x)
        gl = torch.zeros(1, dtype=torch.float64, device="cuda")
        gw = torch.zeros(wl.L, dtype=torch.float64, device="cuda")

        def step():
            S.segsalsa_str_solve_ckpt(pr, ck, x, z, ws)
            S.segsalsa_str_backward(pr, ck, x, gz, gi, ws, gl, gw)

        ms, _ = time_calls(torch, step, steps, warmup)
        ms_fwd, _ = time_calls(torch, lambda: S.segsalsa_str_solve_ckpt(pr, ck, x, z, ws), steps, 1)
        S.segsalsa_profile_read(reset=True)
        S.segsalsa_profile_enable(True)
        S.segsalsa_str_backward(pr, ck, x, gz, gi, ws, gl, gw)
        torch.cuda.synchronize()
        S.segsalsa_profile_enable(False)
        tot = S.segsalsa_profile_read(reset=True)
        adj = tot["adjoint_prox"]
        out[tag] = {"ms_per_step": ms, "ms_forward_ckpt": ms_fwd, "ms_backward": ms - ms_fwd,
                    "value": units / (ms * 1e-3), "backward_over_forward": (ms - ms_fwd) / ms_fwd,
                    "adjoint_prox_avg_us": 1e3 * adj[0] / max(1, adj[1])}
        out[tag + "_grad"] = {"lambda": float(gl.item()), "weights_l2": float(torch.linalg.vector_norm(gw).item()),
                              "input_l2": float(torch.linalg.vector_norm(gi.double()).item())}
        log(f"[bench] adjoint {tag}: {out[tag]}")
        del ws, x, z, gi
        torch.cuda.empty_cache()
    g32, g64 = out["f32_grad"], out["f64_grad"]
    out["grad_rel_err_fp32_vs_fp64"] = {
        "lambda": abs(g32["lambda"] - g64["lambda"]) / abs(g64["lambda"]),
        "weights_l2": abs(g32["weights_l2"] - g64["weights_l2"]) / g64["weights_l2"],
        "input_l2": abs(g32["input_l2"] - g64["input_l2"]) / g64["input_l2"]}
    return out


def bench_variants(S, torch, synth, steps, warmup):
    """The 145x145 workload with the method's variants: g4 as the simplex projection, and the
    general Schatten p (p = 3, per-pixel Newton solve); FP32 throughput and its z error vs FP64."""
    wl = synth.WORKLOADS["pines_145x145_k16"]
    d = synth.make_workload(wl)
    units = wl.n * wl.K * wl.iters
    out = {"workload": wl.name}
    for name, kw in (("g4_simplex", dict(schatten_p=wl.schatten_p, g4_simplex=True)), ("schatten_p3", dict(schatten_p=3.0))):
        zs, rec = {}, {}
        for dtype, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
            x = torch.from_numpy(d["probs"]).to(device="cuda", dtype=dtype)
            pr = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], kw["schatten_p"], wl.lam, wl.mu, wl.iters,
                           g4_simplex=kw.get("g4_simplex", False))
            ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
            z = torch.empty_like(x)
            ms, _ = time_calls(torch, lambda: S.segsalsa_str_solve(pr, x, z, ws), steps, warmup)
            zs[tag] = z.double()
            rec[tag] = {"ms_per_step": ms, "value": units / (ms * 1e-3)}
            del ws, x
        rec["z_err_fp32_vs_fp64"] = float(torch.max(torch.abs(zs["f32"] - zs["f64"])).item())
        out[name] = rec
        log(f"[bench] variant {name}: {rec}")
    return out


def bench_sweep(S, torch, synth, wl_name="pines_145x145_k16", radii=(0, 1, 2, 3, 4, 5), dtype_name="f32",
                iters=None, steps=1):
    """Synthetic analogue of the patch-size experiment (Sec. 5, Fig. 1): patches 1x1 ... 11x11 with
    Gaussian bandwidth gamma = M (the distance from the patch border to its centre; 1 for 1x1),
    argmax labels after the rounds against the Voronoi ground truth, next to argmax p."""
    import dataclasses
    wl = synth.WORKLOADS[wl_name]
    if iters is not None:
        wl = dataclasses.replace(wl, iters=iters)
    d = synth.make_workload(wl)
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    truth = torch.from_numpy(d["labels"]).cuda()
    x = torch.from_numpy(d["probs"]).to(device="cuda", dtype=dtype)
    lab = torch.empty(wl.H, wl.W, dtype=torch.int32, device="cuda")
    S.segsalsa_str_labels(x, lab)
    torch.cuda.synchronize()
    out = {"workload": wl.name, "rounds": wl.iters, "lambda": wl.lam, "mu": wl.mu, "dtype": dtype_name,
           "accuracy_argmax_p": float((lab == truth).float().mean().item()), "patches": []}
    for M in radii:
        gamma = max(M, 1)
        c = synth.gaussian_patch_multipliers(M, float(gamma))
        pr = S.Problem(wl.K, wl.H, wl.W, M, c, wl.schatten_p, wl.lam, wl.mu, wl.iters)
        ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
        z = torch.empty_like(x)
        ms, _ = time_calls(torch, lambda: S.segsalsa_str_solve(pr, x, z, ws), steps, 1)
        S.segsalsa_str_labels(z, lab)
        torch.cuda.synchronize()
        acc = float((lab == truth).float().mean().item())
        L = (2 * M + 1) ** 2
        out["patches"].append({"patch": f"{2 * M + 1}x{2 * M + 1}", "gamma": gamma, "L": L, "accuracy": acc,
                               "ms_per_solve": ms, "value": wl.n * wl.K * wl.iters / (ms * 1e-3)})
        log(f"[bench] sweep {2 * M + 1}x{2 * M + 1}: accuracy {acc:.4f}, {ms:.2f} ms")
        del ws, z
        torch.cuda.empty_cache()
    return out


def plan_record(S, K, H, W, M, prec):
    """The launch shapes of a single-image solve of this shape and whether they came from the tuning table."""
    t, tuned = S.segsalsa_tuning_get(K, H, W, M, prec)
    rec = {k: v for k, v in t.items() if k != "us_per_round"}
    rec["tuned"] = tuned
    return rec


def bench_batch(S, torch, synth, steps, warmup, fp32_only=False, graph=True):
    """The 64-image batch (sides 96..512, K in {4, 8, 9, 16}, 3x3 patch, 200 rounds): one step is
    one segsalsa_str_solve_batch call (one graph launch)."""
    B = synth.BATCH
    shapes = synth.batch_shapes()
    probs = [t[0] for t in synth.make_batch(shapes)]
    c = synth.gaussian_patch_multipliers(B["M"], B["patch_sigma"])
    imgs, total = S.image_table([(K, H, W) for (H, W, K) in shapes], [B["lam"]] * len(shapes),
                                [B["mu"]] * len(shapes))
    units = sum(H * W * K for (H, W, K) in shapes) * B["iters"]
    L = (2 * B["M"] + 1) ** 2
    out, zs = {}, {}
    for dtype, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
        if fp32_only and tag == "f64":
            continue
        packed = torch.cat([torch.from_numpy(x).reshape(-1) for x in probs]).to(device="cuda", dtype=dtype)
        z = torch.empty_like(packed)
        params = S.BatchParams(B["M"], c, 1.0, B["iters"], use_graph=graph)
        ws = torch.empty(S.segsalsa_str_batch_workspace_size(imgs, params, S._prec(dtype)), dtype=torch.uint8,
                         device="cuda")
        log(f"[bench] batch {tag}")
        n_steps, n_warm = (steps, warmup) if tag == "f32" else (max(1, min(2, steps)), 1)
        ms, _ = time_calls(torch, lambda: S.segsalsa_str_solve_batch(imgs, params, packed, z, ws), n_steps, n_warm)
        direct = S.BatchParams(B["M"], c, 1.0, B["iters"])
        ph = phase_times(S, torch, lambda: S.segsalsa_str_solve_batch(imgs, direct, packed, z, ws), 1)
        zs[tag] = z.double()
        out[tag] = dict(ms_per_step=ms, value=units / (ms * 1e-3), phases=ph)
        log(f"[bench] batch {tag}: {ms:.2f} ms/step {units / (ms * 1e-3):.4g} units/s {ph}")
        del ws, packed
        torch.cuda.empty_cache()
    z_err = float(torch.max(torch.abs(zs["f32"] - zs["f64"])).item()) if "f64" in zs else None
    n_units = sum(H * W * K for (H, W, K) in shapes)
    prox = out["f32"]["phases"]["prox_rhs"]   # all prox launches of a round (one per workgroup shape)
    bytes_launch = n_units * prox_bytes_per_unit(L, 4)
    achieved = bytes_launch / (prox["avg_us"] * 1e-6) / 1e9
    round_us = out["f32"]["ms_per_step"] * 1e3 / B["iters"]
    res = {"workload": B["name"], "value": out["f32"]["value"] if (z_err is None or z_err <= Z_TOL) else 0.0,
           "unit": UNIT, "ms_per_step": out["f32"]["ms_per_step"], "steps": steps, "warmup": warmup, "dtype": "f32",
           "config": {"images": len(shapes), "pixels": sum(H * W for H, W, _ in shapes), "units_per_round": n_units,
                      "patch": "3x3", "rounds": B["iters"], "graph": graph},
           "roofline": {"bound": "hbm", "kernel": "prox_rhs (all launches of a round)", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "bytes_per_launch_alg": bytes_launch, "avg_launch_us": prox["avg_us"]},
           "round_roofline": round_roofline(n_units, L, round_us),
           "z_err_fp32_vs_fp64": z_err,
           "phases_f32_us": {k: round(v["avg_us"], 3) for k, v in out["f32"]["phases"].items()},
           "plans": [dict(K=K, H=H, W=W, **{k: v for k, v in t.items() if k != "us_per_round"}, tuned=False)
                     for (H, W, K), t in zip(shapes, S.segsalsa_str_batch_plans(
                         imgs, S.BatchParams(B["M"], c, 1.0, B["iters"]), S.SEGSALSA_FP32))]}
    if "f64" in out:
        res["fp64"] = {"value": out["f64"]["value"], "ms_per_step": out["f64"]["ms_per_step"]}
        res["speedup_fp32_vs_fp64"] = out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"]
    return res


def hbm_copy_rate(torch, nbytes=2 << 30, reps=5):
    """GB/s (read + write) of a plain device-to-device copy of nbytes (torch's copy kernel): the
    streaming rate a read-modify-write kernel can expect on this GPU, next to the 8 TB/s peak."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def hbm_stream_rate(S, torch, nbytes=2 << 30, reps=5):
    """GB/s (read + write) of the library's streaming copy of nbytes (16-byte nontemporal loads and stores,
    the access pattern of the prox kernel's streaming build): the practical ceiling of that kernel."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    S.segsalsa_stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        S.segsalsa_stream_copy(src, dst)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def round_roofline(n_units, L, round_us, b=4):
    """Whole round (prox + the three FFT passes) against HBM: (4L + 15) words per pixel*class,
    the prox kernel's (4L + 9) plus the FFT passes' right-hand side and two spectrum round trips."""
    achieved = n_units * (4 * L + 15) * b / (round_us * 1e-6) / 1e9
    return {"bound": "hbm", "bytes_per_unit": (4 * L + 15) * b, "us_per_round": round_us, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_2048x2048_k16")
    ap.add_argument("--rounds", type=int, default=None,
                    help="override the workload's round count (profiler runs; the line then is not the headline)")
    ap.add_argument("--schatten-p", type=float, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable-solve measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-image batch entry")
    ap.add_argument("--no-variants", action="store_true", help="skip the simplex-g4 / general-p measurement")
    ap.add_argument("--sweep", action="store_true",
                    help="patch-size sweep 1x1 ... 11x11 on the workload (accuracy vs the synthetic ground truth)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the differentiable solve (forward with checkpoints + reverse sweep)")
    ap.add_argument("--fp32-only", action="store_true", help="time only the FP32 path (for profiler runs)")
    ap.add_argument("--no-graph", action="store_true", help="launch the kernels directly instead of one graph")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on every single-image workload shape in FP32 and FP64 and write the "
                         "package's tuning cache")
    ap.add_argument("--tune-rounds", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain copy of known size, 512 MiB FP32 read from an evicted source "
                         "and 256 MiB BF16 written (reference for the HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (the solver "
              "shards nothing across GPUs).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1504_07028_amd import segsalsa as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    S.lib()

    if args.calibrate_copy:
        # a plain copy of known size for the HBM counters: 512 MiB of FP32 read and written as
        # 256 MiB of BF16 (its own kernel, named by the BF16 output type), from a source that 2 GiB
        # written in between has evicted from the L2s and the 256 MB MALL
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        flush = torch.empty(512 * 1024 * 1024, dtype=torch.float32, device="cuda")
        flush.fill_(2.0)
        torch.cuda.synchronize()
        dst = src.to(torch.bfloat16)
        torch.cuda.synchronize()
        log("[bench] calibration copy (FP32 -> BF16): 536870912 bytes read, 268435456 bytes written")
        del src, dst, flush

    if args.sweep:
        print(json.dumps(bench_sweep(S, torch, synth, args.workload, steps=args.steps)), flush=True)
        return

    if args.tune:
        from paper_1504_07028_amd import autotune
        # single-image workloads only: batches of several images keep the planner's shapes
        shapes = [(w.K, w.H, w.W, w.M) for w in synth.WORKLOADS.values()]
        t0 = time.perf_counter()
        res = autotune.tune_shapes(shapes, ["fp32", "fp64"], args.tune_rounds, S.DEFAULT_TUNING_CACHE, fresh=True,
                                   log=log)
        print(json.dumps({"tuned": len(res), "seconds": time.perf_counter() - t0,
                          "cache": os.path.relpath(S.DEFAULT_TUNING_CACHE, ROOT)}), flush=True)
        return

    if args.adjoint_only:
        print(json.dumps(bench_adjoint(S, torch, synth, args.steps, args.warmup)), flush=True)
        return

    if args.workload == synth.BATCH["name"]:
        print(json.dumps(bench_batch(S, torch, synth, args.steps, args.warmup, args.fp32_only, not args.no_graph)),
              flush=True)
        return

    import dataclasses
    wl = synth.WORKLOADS[args.workload]
    if args.schatten_p is not None:
        wl = dataclasses.replace(wl, schatten_p=args.schatten_p)
    if args.rounds is not None:
        wl = dataclasses.replace(wl, iters=args.rounds)
    d = synth.make_workload(wl)
    units = wl.n * wl.K * wl.iters
    res = {}
    zs = {}
    for dtype, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
        if args.fp32_only and tag == "f64":
            continue
        x = torch.from_numpy(d["probs"]).to(device="cuda", dtype=dtype)
        pr = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], wl.schatten_p, wl.lam, wl.mu, wl.iters,
                       use_graph=not args.no_graph)
        ws = torch.empty(S.segsalsa_str_workspace_size(pr, S._prec(dtype)), dtype=torch.uint8, device="cuda")
        z = torch.empty_like(x)
        # FP64 is timed over at most two solves (no warm-up: it is the reference for the error gate)
        n_steps, n_warm = (args.steps, args.warmup) if tag == "f32" else (max(1, min(2, args.steps)), 0)
        log(f"[bench] {wl.name} {tag}: warmup {n_warm}, steps {n_steps}, graph {not args.no_graph}")
        ms_gpu, ms_wall = time_calls(torch, lambda: S.segsalsa_str_solve(pr, x, z, ws), n_steps, n_warm)
        zs[tag] = z.double().cpu().numpy()
        phases = None
        if tag == "f32":
            # per-kernel durations: one more solve, direct launches with HIP events around each
            # launch, recorded on the solve's stream
            pr_direct = S.Problem(wl.K, wl.H, wl.W, wl.M, d["weights"], wl.schatten_p, wl.lam, wl.mu, wl.iters)
            phases = phase_times(S, torch, lambda: S.segsalsa_str_solve(pr_direct, x, z, ws), 1)
        res[tag] = dict(ms_per_step=ms_gpu, ms_wall=ms_wall, value=units / (ms_gpu * 1e-3), phases=phases,
                        plan=plan_record(S, wl.K, wl.H, wl.W, wl.M, S._prec(dtype)))
        log(f"[bench] {tag}: {ms_gpu:.3f} ms/step, {units / (ms_gpu * 1e-3):.4g} units/s, phases {phases}")
        del ws, x, z
        torch.cuda.empty_cache()

    z_err = float(np.max(np.abs(zs["f32"] - zs["f64"]))) if "f64" in zs else None
    b = 4
    prox = res["f32"]["phases"]["prox_rhs"]
    bytes_launch = wl.n * wl.K * prox_bytes_per_unit(wl.L, b)
    achieved = bytes_launch / (prox["avg_us"] * 1e-6) / 1e9
    src_hash = kernel_source_hash()
    traffic = load_traffic(wl.name, "f32", src_hash)
    copy_gbs = hbm_copy_rate(torch)
    stream_gbs = hbm_stream_rate(S, torch)
    value = res["f32"]["value"] if (z_err is None or z_err <= Z_TOL) else 0.0
    round_us = res["f32"]["ms_per_step"] * 1e3 / max(1, wl.iters)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["f32"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "H": wl.H, "W": wl.W, "K": wl.K, "patch": f"{2 * wl.M + 1}x{2 * wl.M + 1}",
                   "schatten_p": wl.schatten_p, "lambda": wl.lam, "mu": wl.mu, "rounds": wl.iters,
                   "graph": not args.no_graph, "plan": res["f32"]["plan"]},
        "roofline": {"bound": "hbm", "kernel": "prox_rhs", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch_alg": bytes_launch,
                     "avg_launch_us": prox["avg_us"], "kernel_source_hash": src_hash,
                     "frac_of_copy": achieved / copy_gbs, "frac_of_stream_copy": achieved / stream_gbs},
        "round_roofline": round_roofline(wl.n * wl.K, wl.L, round_us),
        "z_err_fp32_vs_fp64": z_err,
        "hbm_copy_gbs": copy_gbs,
        "hbm_stream_copy_gbs": stream_gbs,
        "phases_f32_us": {k: round(v["avg_us"], 3) for k, v in res["f32"]["phases"].items()},
    }
    if "f64" in res:
        out["fp64"] = {"value": res["f64"]["value"], "ms_per_step": res["f64"]["ms_per_step"],
                       "plan": res["f64"]["plan"]}
        out["speedup_fp32_vs_fp64"] = res["f64"]["ms_per_step"] / res["f32"]["ms_per_step"]
    if not args.no_batch:
        out["batch"] = bench_batch(S, torch, synth, args.steps, args.warmup, args.fp32_only, not args.no_graph)
    if not args.no_adjoint and not args.fp32_only:
        out["adjoint"] = bench_adjoint(S, torch, synth, 2, 1)
    if not args.fp32_only and not args.no_variants:
        out["variants"] = bench_variants(S, torch, synth, 2, 1)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, d["probs"], d["weights"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
