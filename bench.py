#!/usr/bin/env python3
"""Throughput of the FasterTucker hot path on one MI355X.

A step is one iteration of Algorithm 2 (the factor pass of every mode and the
core pass of every mode, each followed by its C refresh) plus the RMSE pass.
The metric counts 2 N |Omega| element updates per step (one factor and one
core visit per element and mode).

Default run (the metric: FP32 against BF16 storage at matched RMSE, and the
fraction of the roofline): the Netflix-shaped synthetic tensor at the ranks of
the paper's Table 5 (480000 x 18000 x 2200, 100M distinct coordinates with
per-mode Zipf(1.1) indices, integer values 1..5, J = R = 32), timed once with
FP32 storage and once with BF16 storage (FP32 masters and arithmetic); the
line's value is the BF16 leg.  Beside it: the held-out RMSE of FP32 and BF16
after the same iterations on a planted tensor that the model can learn
(matched RMSE), and the same tensor at J = R = 16 in FP32.  `--workload`
selects a single workload and storage instead (sweeps, ablations).

Prints one JSON line.  The inputs are generated and uploaded before the timed
region; the timed region holds only device work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (published)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def algorithmic(w, nnz, row_counts, heads, fibers, relaxed=False, sp=4):
    """Per-epoch algorithmic flops and bytes per kernel family (formulas in the design notes).

    fibers[m] is the number of mode-m fibers when g = B(m) w is shared per fiber
    (Section 3.2), else None: a shared mode computes g once per fiber and the
    factor kernels read it instead of forming it per element.  With relaxed
    factor passes the chunk kernel runs the plain SGD steps (no map matrix).
    sp: bytes per stored parameter (4 FP32, 2 BF16): the size of the C and A
    tables the kernels read; the factor pass reads and writes the FP32 masters.
    """
    import numpy as np

    N, J, R = len(w.dims), w.J[0], w.R
    stream = (N - 1) * 4 + 4
    out = {"factor_compose": [0.0, 0.0], "factor_apply": [0.0, 0.0], "fiber_g": [0.0, 0.0], "segsum": [0.0, 0.0],
           "loss": [0.0, 0.0], "compose_executed": [0.0, 0.0], "factor_fused": [0.0, 0.0],
           "fused_executed": [0.0, 0.0]}
    c_bytes = [d * R * sp for d in w.dims]
    a_bytes = [d * J * 4 for d in w.dims]
    a_read = [d * J * sp for d in w.dims]
    for m in range(N):
        L = row_counts[m]
        head = heads[m]
        heavy = L > head
        comp = float(np.sum(np.where(heavy, L - head, 0)))
        app = float(nnz - comp)
        others = sum(c_bytes) - c_bytes[m]
        if fibers[m] is None:
            f_elem = 2 * J * R + (N - 2) * R + 5 * J
            e_bytes = stream
            c_share = others
        else:
            # g per fiber: w (N-2 products of R), g = B w (2 J R); the factor
            # kernels then stream the fiber id and read g (J floats).
            nf = fibers[m]
            out["fiber_g"][0] += nf * (2 * J * R + (N - 2) * R)
            out["fiber_g"][1] += nf * ((N - 1) * 4 + J * 4) + others
            f_elem = 5 * J
            e_bytes = 4 + 4 + J * 4
            c_share = 0.0
        out["factor_compose"][0] += comp * f_elem
        # executed on top: the chunk map's matrix part, a J x J matrix-vector
        # product and a rank-1 update per element (4 J^2 flops)
        out["compose_executed"][0] += comp * (f_elem + (2 * J if relaxed else 4 * J * J))
        out["factor_compose"][1] += comp * e_bytes + c_share * comp / max(nnz, 1)
        out["factor_apply"][0] += app * f_elem
        out["factor_apply"][1] += app * e_bytes + c_share * app / max(nnz, 1) + 2 * a_bytes[m]
        out["segsum"][0] += nnz * ((N - 2) * R + 4 * R) + w.dims[m] * 2 * J * R
        out["segsum"][1] += nnz * stream + others + c_bytes[m] + a_read[m]
    out["loss"][0] += nnz * (N * R + 3)
    out["loss"][1] += nnz * stream + sum(c_bytes)
    # the exact passes launch the in-place items and the chunk maps as one kernel
    for k in (0, 1):
        out["factor_fused"][k] = out["factor_compose"][k] + out["factor_apply"][k]
    out["fused_executed"][0] = out["compose_executed"][0] + out["factor_apply"][0]
    return out


def cpu_baseline(w, c, v, A, B, sample):
    """The FP64 oracle, as it is, on the first `sample` elements of the same tensor (one thread)."""
    import numpy as np

    import oracle

    cs = np.ascontiguousarray(c[:, :sample])
    vs = v[:sample].astype(np.float64)
    orc = oracle.Model(w.dims, w.J, w.R, cs, vs, [a.astype(np.float64) for a in A], [b.astype(np.float64) for b in B])
    t = time.perf_counter()
    orc.epoch(w.lr, w.lam, w.lr, w.lam)
    orc.loss()
    dt = time.perf_counter() - t
    N = len(w.dims)
    return {
        "value": 2 * N * sample / dt,
        "unit": "nnz-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one epoch + RMSE of the FP64 C oracle on the first {sample} elements of the same tensor "
        f"(same dims, J, R), {dt:.2f} s",
    }


COUNTER_FILES = {("netflix32", "f32"): "profiles/netflix32_fp32_hbm_counters.md",
                 ("netflix32", "bf16"): "profiles/netflix32_bf16_hbm_counters.md"}
KERNEL_SOURCES = ["ft_device.h", "ft_refresh.hip", "ft_factor.hip", "ft_segment.hip"]


def kernel_sources_sha256():
    """sha256 over the device sources, in KERNEL_SOURCES order (recorded with the counter summaries)."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2210_06014_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def counter_traffic(workload, storage, kernel):
    """Measured HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when
    there is none for this workload and storage or the kernel source has changed since the counters were
    taken."""
    import re

    path = COUNTER_FILES.get((workload, storage))
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    m = re.search(r"<!-- traffic-data (.*?) -->", open(os.path.join(ROOT, path)).read())
    if not m:
        return None
    data = json.loads(m.group(1))
    if kernel_sources_sha256() != data.get("kernels_sha256"):
        return None
    return data["traffic_bytes_per_launch"].get(kernel)


def copy_calibration(nbytes):
    """A plain copy kernel of known size: what FETCH_SIZE / WRITE_SIZE read for it calibrates the counters."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 3
    print(json.dumps({"copy_bytes": nbytes, "ms_per_copy": ms, "GBps_read_plus_write": 2 * nbytes / ms / 1e6}),
          flush=True)


def curve(args):
    """Convergence run (the analogue of the paper's Figure 3): train on 90 % of a planted tensor, report the
    training RMSE and the held-out RMSE and MAE after every iteration, one JSON line each."""
    import numpy as np
    import torch

    import paper_2210_06014_amd as ft
    import synth

    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    nnz = w.nnz if args.nnz is None else args.nnz
    lr = w.lr if args.lr is None else args.lr
    c, v, A, B = synth.make(w, nnz=nnz)
    test = synth.test_mask(nnz, w.seed)
    ctr, vtr = np.ascontiguousarray(c[:, ~test]), np.ascontiguousarray(v[~test])
    cte = torch.from_numpy(np.ascontiguousarray(c[:, test])).cuda()
    vte = v[test].astype(np.float64)
    N, J, R = len(w.dims), w.J[0], w.R
    plan = ft.Plan(w.dims, J, R, ctr, vtr, chunk=args.chunk, head=args.head, relaxed=args.relaxed)
    prm = ft.Params(A, B, storage=args.storage)
    ft.refresh(plan, prm)

    def report(epoch, ms):
        train = float(ft.loss(plan, prm)[1].item())
        xh = ft.predict(plan, prm, cte).double().cpu().numpy()
        err = xh - vte
        line = {"epoch": epoch, "storage": args.storage, "relaxed": args.relaxed, "train_rmse": train,
                "test_rmse": float(np.sqrt(np.mean(err * err))), "test_mae": float(np.mean(np.abs(err))),
                "ms_per_iteration": ms}
        print(json.dumps(line), flush=True)
        return line

    report(0, 0.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    last = None
    for ep in range(1, args.curve + 1):
        e0.record()
        ft.epoch(plan, prm, lr, w.lam, lr, w.lam)
        e1.record()
        torch.cuda.synchronize()
        last = report(ep, e0.elapsed_time(e1))
    summary = {"curve": args.workload, "storage": args.storage, "relaxed": args.relaxed, "epochs": args.curve, "train_elements": int(vtr.size),
               "test_elements": int(vte.size), "lr": lr, "lam": w.lam, "sigma": w.sigma, "J": J, "R": R,
               "final_test_rmse": last["test_rmse"], "final_test_mae": last["test_mae"],
               "test_rmse_of_the_mean": float(np.sqrt(np.mean((vte - vtr.mean()) ** 2)))}
    print(json.dumps(summary), flush=True)




def time_steps(ft, plan, prm, w, steps, warmup, profile=True):
    """W untimed steps, then `steps` timed steps (iteration + RMSE pass) between two synchronisations.
    Returns (ms per step, per-kernel timing or {}, RMSE before the warm-up, RMSE after the timed steps)."""
    import torch

    rmse0 = float(ft.loss(plan, prm)[1].item())
    lossbuf = torch.empty(4, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
        ft.loss(plan, prm, out=lossbuf)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
        ft.loss(plan, prm, out=lossbuf)
    ev1.record()
    torch.cuda.synchronize()
    prof = plan.profile_read() if profile else {}
    plan.profile(False)
    return ev0.elapsed_time(ev1) / steps, prof, rmse0, float(lossbuf[1].item())


def time_passes(ft, plan, prm, w, steps):
    """The per-pass measures of the paper's Table 5: N |Omega| / wall time of the factor epoch (N factor passes
    with their C refreshes and shared-g passes) and of the core epoch, timed apart on extra steps."""
    import torch

    N, nnz = plan.order, plan.nnz
    f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t_f = t_c = 0.0
    for _ in range(steps):
        f0.record()
        ft.factor_epoch(plan, prm, w.lr, w.lam)
        f1.record()
        ft.core_epoch(plan, prm, w.lr, w.lam)
        f2.record()
        torch.cuda.synchronize()
        t_f += f0.elapsed_time(f1) / steps
        t_c += f1.elapsed_time(f2) / steps
    return {"factor_ms": t_f, "core_ms": t_c, "factor_nnz_per_s": N * nnz / (t_f / 1e3),
            "core_nnz_per_s": N * nnz / (t_c / 1e3),
            "factor_core_nnz_updates_per_s": 2 * N * nnz / ((t_f + t_c) / 1e3),
            "note": "wall time of factor_epoch and core_epoch calls, timed apart after the measured steps"}


def rooflines(w, nnz, c, plan, prof, steps, storage, relaxed, counters_ok):
    """Per-kernel rates, the roofline object of the dominant kernel and that of the core gather pass."""
    import numpy as np

    N = len(w.dims)
    counts = [np.bincount(c[m], minlength=w.dims[m]) for m in range(N)]
    infos = [plan.mode_info(m) for m in range(N)]
    fibers = [info["fibers"] if info["fiber_shared"] else None for info in infos]
    heads = [info["head"] for info in infos]
    alg = algorithmic(w, nnz, counts, heads, fibers, relaxed, sp=2 if storage == "bf16" else 4)
    kernels = {}
    for k, (ms, n) in prof.items():
        if n:
            kernels[k] = {"ms_per_step": ms / steps, "launches_per_step": n / steps, "avg_launch_us": 1e3 * ms / n}

    def obj(k):
        t_s = kernels[k]["ms_per_step"] / 1e3
        flops, byts = alg.get(k, [0.0, 0.0])
        launches = kernels[k]["launches_per_step"]
        traffic = counter_traffic(w.name, storage, k) if counters_ok else None
        if k in ("factor_compose", "factor_apply", "factor_fused"):
            ach = flops / t_s / 1e12
            r = {"kernel": k, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                 "frac": ach / PEAK_FP32_TFLOPS, "traffic": traffic, "algorithmic_per_launch": flops / launches,
                 "algorithmic_bytes_per_launch": byts / launches, "avg_launch_us": kernels[k]["avg_launch_us"]}
            if k in ("factor_compose", "factor_fused"):
                exk = "compose_executed" if k == "factor_compose" else "fused_executed"
                ex = alg[exk][0] / t_s / 1e12
                r.update({"executed_per_launch": alg[exk][0] / launches, "executed_achieved": ex,
                          "executed_frac": ex / PEAK_FP32_TFLOPS})
            return r
        ach = byts / t_s / 1e9
        r = {"kernel": k, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "algorithmic_per_launch": byts / launches,
             "avg_launch_us": kernels[k]["avg_launch_us"]}
        if k in ("segsum", "loss"):
            # the bytes against HBM are the stream; the gathered C rows come through the caches, and
            # the CU's vector-memory data path is what saturates (rocprofv3 TD/TA busy counters)
            r["limiter"] = ("vector-memory data path of the CUs (TD 92-95 % busy, TA 84-90 %), "
                            "profiles/netflix32_fp32_segment_pass_limiter.md")
        return r

    dom = gather = None
    if kernels:
        dom = obj(max(kernels, key=lambda k: kernels[k]["ms_per_step"]))
        if "segsum" in kernels:
            gather = obj("segsum")
    for k in kernels:
        if k in alg and k not in ("compose_executed", "fused_executed"):
            t_k = kernels[k]["ms_per_step"] / 1e3
            kernels[k]["alg_tflops"] = alg[k][0] / t_k / 1e12
            kernels[k]["alg_gbs"] = alg[k][1] / t_k / 1e9
    return kernels, dom, gather, infos, fibers


def leg(ft, w, c, plan, A, B, storage, args, nnz, relaxed=False):
    """One storage form on one plan: timed steps, per-kernel rooflines, per-pass throughputs."""
    prm = ft.Params(A, B, storage=storage)
    ft.refresh(plan, prm)
    ms, prof, rmse0, rmse = time_steps(ft, plan, prm, w, args.steps, args.warmup, not args.no_profile)
    log(f"{w.name} {storage}: {ms:.3f} ms/step, RMSE {rmse0:.7f} -> {rmse:.7f}")
    counters_ok = (args.nnz is None and not args.chunk and not args.head and not args.no_fiber_share
                   and not args.no_c_cache and not relaxed and not args.split_factor and not args.run_reuse)
    kernels, dom, gather, infos, fibers = rooflines(w, nnz, c, plan, prof, args.steps, storage, relaxed,
                                                    counters_ok)
    passes = time_passes(ft, plan, prm, w, args.steps)
    N = len(w.dims)
    return {"storage": storage, "value": 2 * N * nnz / (ms / 1e3), "ms_per_step": ms, "rmse_start": rmse0,
            "rmse_end": rmse, "roofline": dom, "roofline_gather": gather, "passes": passes, "kernels": kernels,
            "fiber_shared_modes": [m for m in range(N) if fibers[m] is not None],
            "fibers_per_mode": [info["fibers"] for info in infos],
            "heads_per_mode": [info["head"] for info in infos], "chunk": infos[0]["chunk"]}


def describe(w, nnz):
    return (f"{w.name}: {'x'.join(map(str, w.dims))}, {nnz} distinct coordinates, Zipf({w.zipf}) per mode, "
            f"values {w.value_kind}, J={w.J[0]}, R={w.R}, lr={w.lr}, lam={w.lam}, init N(0,{w.sigma}^2)")


def planted_match(ft, iters):
    """Matched RMSE in a learning regime: the planted tensor (10 % held out), FP32 and BF16 storage from the
    same initial parameters, held-out RMSE after each of `iters` iterations."""
    import numpy as np
    import torch

    import synth

    w = synth.WORKLOADS["planted"]
    c, v, A, B = synth.make(w)
    test = synth.test_mask(w.nnz, w.seed)
    ctr, vtr = np.ascontiguousarray(c[:, ~test]), np.ascontiguousarray(v[~test])
    cte = torch.from_numpy(np.ascontiguousarray(c[:, test])).cuda()
    vte = v[test].astype(np.float64)
    plan = ft.Plan(w.dims, w.J[0], w.R, ctr, vtr)
    curves = {}
    for storage in ("f32", "bf16"):
        prm = ft.Params(A, B, storage=storage)
        ft.refresh(plan, prm)
        rm = []
        for _ in range(iters):
            ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
            err = ft.predict(plan, prm, cte).double().cpu().numpy() - vte
            rm.append(float(np.sqrt(np.mean(err * err))))
        curves[storage] = rm
    rel = [abs(b - f) / f for f, b in zip(curves["f32"], curves["bf16"])]
    k = int(np.argmax(rel))
    out = {"workload": describe(w, w.nnz) + "; planted separable values, 10 % held out",
           "iterations": iters, "test_rmse_f32": curves["f32"][-1], "test_rmse_bf16": curves["bf16"][-1],
           "final_rel_diff": rel[-1], "max_rel_diff": rel[k], "max_rel_diff_at_iteration": k + 1,
           "test_rmse_f32_per_iteration": curves["f32"], "test_rmse_bf16_per_iteration": curves["bf16"],
           "test_rmse_of_the_mean": float(np.sqrt(np.mean((vte - vtr.mean()) ** 2)))}
    log(f"planted: test RMSE after {iters} iterations f32 {curves['f32'][-1]:.5f} bf16 {curves['bf16'][-1]:.5f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=None,
                    help="one workload and storage (default: the metric run, netflix32 FP32 and BF16 legs)")
    ap.add_argument("--nnz", type=int, default=None, help="override the element count (smaller test runs)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="elements of the oracle's CPU sample (default: 12M at J = R = 16, scaled by (16/J)^2: "
                    "about 15 s of oracle time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-planted", action="store_true", help="metric run without the matched-RMSE curves")
    ap.add_argument("--planted-iters", type=int, default=20)
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--chunk", type=int, default=0, help="elements per chunk map of a long row (0: library default)")
    ap.add_argument("--head", type=int, default=0,
                    help="rows longer than this are split into a head and chunks (0: library default)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16"],
                    help="parameter storage with --workload: FP32, or BF16 copies with FP32 masters and arithmetic")
    ap.add_argument("--no-fiber-share", action="store_true",
                    help="form g = B(m) w per element instead of once per mode-m fiber (Section 3.2 ablation)")
    ap.add_argument("--no-c-cache", action="store_true",
                    help="factor and core passes form C rows from A and B on use (FastTucker's cost; Table 5 ablation)")
    ap.add_argument("--split-factor", action="store_true",
                    help="launch the in-place items and the chunk maps of the exact factor passes as two kernels "
                    "(FT_SPLIT_FACTOR; the layout before fusing them)")
    ap.add_argument("--run-reuse", action="store_true",
                    help="segment passes gather the C row of mode m + 1 once per run of elements sharing it "
                    "(FT_RUN_REUSE; fewer gathers, measured slower)")
    ap.add_argument("--relaxed", action="store_true",
                    help="relaxed factor passes: chunks of long rows start from the row as its head left it and "
                    "their increments are merged with a step guard (FT_RELAXED)")
    ap.add_argument("--curve", type=int, default=0,
                    help="convergence run instead of the benchmark: this many iterations on a planted tensor "
                    "(e.g. --workload planted), printing train RMSE and held-out RMSE/MAE per iteration")
    ap.add_argument("--lr", type=float, default=None, help="learning rate of a convergence run (default: workload's)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_bytes:
        return copy_calibration(args.copy_bytes)
    if args.curve:
        args.workload = args.workload or "planted"
        return curve(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            json.dumps({"error": "the library runs on one GPU only; sharding across GPUs is not implemented",
                        "n_gpus": args.gpus}),
            flush=True,
        )
        sys.exit(2)

    import torch

    import paper_2210_06014_amd as ft
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}), flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    metric_run = args.workload is None
    w = synth.WORKLOADS[args.workload or "netflix32"]
    nnz = w.nnz if args.nnz is None else args.nnz
    N, J, R = len(w.dims), w.J[0], w.R

    log(f"generating {w.name}: dims={w.dims} nnz={nnz} zipf={w.zipf}")
    t = time.time()
    c, v, A, B = synth.make(w, nnz=nnz)
    log(f"generated in {time.time() - t:.1f} s")
    t = time.time()
    plan = ft.Plan(w.dims, J, R, c, v, chunk=args.chunk, head=args.head, fiber_share=not args.no_fiber_share,
                   c_cache=not args.no_c_cache, relaxed=args.relaxed, fused=not args.split_factor,
                   run_reuse=args.run_reuse)
    log(f"plan built and uploaded in {time.time() - t:.1f} s ({plan.device_bytes / 2**30:.2f} GiB plan, "
        f"{plan.scratch_bytes / 2**20:.1f} MiB scratch per parameter set)")

    storages = ["f32", "bf16"] if metric_run else [args.storage]
    legs = {s: leg(ft, w, c, plan, A, B, s, args, nnz, args.relaxed) for s in storages}
    main_leg = legs["bf16" if metric_run else args.storage]

    extra = {}
    if metric_run:
        if not args.no_planted:
            extra["matched_rmse"] = planted_match(ft, args.planted_iters)
        # the same tensor at J = R = 16 (FP32): a second plan for the other ranks
        w16 = synth.WORKLOADS["netflix"]
        del plan
        torch.cuda.empty_cache()
        A16, B16 = synth.init_params(w16.dims, w16.J, w16.R, w16.sigma, w16.seed + 1)
        plan16 = ft.Plan(w16.dims, w16.J[0], w16.R, c, v)
        l16 = leg(ft, w16, c, plan16, A16, B16, "f32", args, nnz)
        extra["netflix_j16_f32"] = {"workload": describe(w16, nnz), **l16}
        del plan16

    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample or int(12_000_000 * (16 / max(J, 16)) ** 2)
        s = min(sample, nnz)
        log(f"CPU baseline: oracle on {s} elements")
        cpu = cpu_baseline(w, c, v, A, B, s)
        log(f"CPU baseline {cpu['value']:.3e} nnz-updates/s")

    bf16 = main_leg["storage"] == "bf16"
    line = {
        "metric": "SGD nnz updates/sec (factor+core)",
        "value": main_leg["value"],
        "unit": "nnz-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 storage, f32 arithmetic" if bf16 else "f32",
        "data": "synthetic",
        "config": {
            "workload": describe(w, nnz),
            "storage": "BF16 copies of A, B, C with FP32 masters and accumulation, FP64 RMSE reduction" if bf16
            else "FP32",
            "step": "factor pass + C refresh per mode, core pass + C refresh per mode, RMSE pass",
            "factor_passes": ("relaxed: chunks of long rows start from the row as its head left it, guarded merge"
                              if args.relaxed else "exact serial SGD per row"),
            "fiber_shared_modes": main_leg["fiber_shared_modes"],
            "fibers_per_mode": main_leg["fibers_per_mode"],
            "heads_per_mode": main_leg["heads_per_mode"],
            "chunk": main_leg["chunk"],
            "rmse_start": main_leg["rmse_start"],
            "rmse_end": main_leg["rmse_end"],
        },
        "roofline": main_leg["roofline"],
        "roofline_gather": main_leg["roofline_gather"],
        "cpu_baseline": cpu,
        "legs": {s: {k: v_ for k, v_ in l.items() if k not in ("fiber_shared_modes", "fibers_per_mode")}
                 for s, l in legs.items()},
        **extra,
    }
    if metric_run:
        f32v, bfv = legs["f32"]["value"], legs["bf16"]["value"]
        line["bf16_vs_f32"] = {"speedup": bfv / f32v, "rmse_end_rel_diff":
                               abs(legs["bf16"]["rmse_end"] - legs["f32"]["rmse_end"]) / legs["f32"]["rmse_end"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
