#!/usr/bin/env python3
"""Throughput of the FasterTucker hot path on one MI355X.

A step is one iteration of Algorithm 2 on a Netflix-shaped synthetic tensor
(480000 x 18000 x 2200, 100M distinct coordinates with per-mode Zipf(1.1)
indices, integer values 1..5, J = R = 16, FP32): the factor pass of every
mode and the core pass of every mode, each followed by its C refresh, then
the RMSE pass.  The metric counts 2 N |Omega| element updates per step
(one factor and one core visit per element and mode).

Prints one JSON line.  The inputs are generated and uploaded before the
timed region; the timed region holds only device work.
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


def algorithmic(w, nnz, row_counts, head, fibers, relaxed=False):
    """Per-epoch algorithmic flops and bytes per kernel family (formulas in the design notes).

    fibers[m] is the number of mode-m fibers when g = B(m) w is shared per fiber
    (Section 3.2), else None: a shared mode computes g once per fiber and the
    factor kernels read it instead of forming it per element.  With relaxed
    factor passes the chunk kernel runs the plain SGD steps (no map matrix).
    """
    import numpy as np

    N, J, R = len(w.dims), w.J[0], w.R
    stream = (N - 1) * 4 + 4
    out = {"factor_compose": [0.0, 0.0], "factor_apply": [0.0, 0.0], "fiber_g": [0.0, 0.0], "segsum": [0.0, 0.0],
           "loss": [0.0, 0.0], "compose_executed": [0.0, 0.0]}
    c_bytes = [d * R * 4 for d in w.dims]
    a_bytes = [d * J * 4 for d in w.dims]
    for m in range(N):
        L = row_counts[m]
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
        out["segsum"][1] += nnz * stream + others + c_bytes[m] + a_bytes[m]
    out["loss"][0] += nnz * (N * R + 3)
    out["loss"][1] += nnz * stream + sum(c_bytes)
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


COUNTER_FILES = {"netflix": "profiles/netflix_j16_fp32_hbm_counters.md"}
KERNEL_SOURCES = ["ft_device.h", "ft_refresh.hip", "ft_factor.hip", "ft_segment.hip"]


def kernel_sources_sha256():
    """sha256 over the device sources, in KERNEL_SOURCES order (recorded with the counter summaries)."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2210_06014_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def counter_traffic(workload, kernel):
    """Measured HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when
    there is none for this workload or the kernel source has changed since the counters were taken."""
    import re

    path = COUNTER_FILES.get(workload)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="netflix")
    ap.add_argument("--nnz", type=int, default=None, help="override the element count (smaller test runs)")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--chunk", type=int, default=0, help="elements per chunk map of a long row (0: library default)")
    ap.add_argument("--head", type=int, default=0,
                    help="rows longer than this are split into a head and chunks (0: library default)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16"],
                    help="parameter storage: FP32, or BF16 copies with FP32 masters and accumulation")
    ap.add_argument("--no-fiber-share", action="store_true",
                    help="form g = B(m) w per element instead of once per mode-m fiber (Section 3.2 ablation)")
    ap.add_argument("--no-c-cache", action="store_true",
                    help="factor and core passes form C rows from A and B on use (FastTucker's cost; Table 5 ablation)")
    ap.add_argument("--relaxed", action="store_true",
                    help="relaxed factor passes: chunks of long rows read the row as it was at the start of the "
                    "pass and their increments are merged with a step guard (FT_RELAXED)")
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
        return curve(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            json.dumps({"error": "the library runs on one GPU only; sharding across GPUs is not implemented",
                        "n_gpus": args.gpus}),
            flush=True,
        )
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2210_06014_amd as ft
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}), flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    nnz = w.nnz if args.nnz is None else args.nnz
    N, J, R = len(w.dims), w.J[0], w.R

    log(f"generating {args.workload}: dims={w.dims} nnz={nnz} zipf={w.zipf}")
    t = time.time()
    c, v, A, B = synth.make(w, nnz=nnz)
    log(f"generated in {time.time() - t:.1f} s")
    t = time.time()
    plan = ft.Plan(w.dims, J, R, c, v, chunk=args.chunk, head=args.head, fiber_share=not args.no_fiber_share,
                   c_cache=not args.no_c_cache, relaxed=args.relaxed)
    log(f"plan built and uploaded in {time.time() - t:.1f} s ({plan.device_bytes / 2**30:.2f} GiB on device)")
    prm = ft.Params(A, B, storage=args.storage)
    ft.refresh(plan, prm)
    rmse0 = float(ft.loss(plan, prm)[1].item())
    lossbuf = torch.empty(4, dtype=torch.float64, device="cuda")

    for i in range(args.warmup):
        ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
        ft.loss(plan, prm, out=lossbuf)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    if not args.no_profile:
        plan.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
        ft.loss(plan, prm, out=lossbuf)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    prof = plan.profile_read() if not args.no_profile else {}
    plan.profile(False)
    ms_step = total_ms / args.steps
    rmse = float(lossbuf[1].item())
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, RMSE {rmse0:.6f} -> {rmse:.6f}")

    value = 2 * N * nnz / (ms_step / 1e3)
    counts = [np.bincount(c[m], minlength=w.dims[m]) for m in range(N)]
    infos = [plan.mode_info(m) for m in range(N)]
    fibers = [info["fibers"] if info["fiber_shared"] else None for info in infos]
    alg = algorithmic(w, nnz, counts, args.head or 2 * (args.chunk or 512), fibers, args.relaxed)
    kernels = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        kernels[k] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps, "avg_launch_us": 1e3 * ms / n}
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        t_s = kernels[dom]["ms_per_step"] / 1e3
        flops, byts = alg.get(dom, [0.0, 0.0])
        traffic = (counter_traffic(args.workload, dom)
                   if args.nnz is None and not args.chunk and not args.head and args.storage == "f32"
                   and not args.no_fiber_share and not args.no_c_cache and not args.relaxed
                   else None)
        launches = kernels[dom]["launches_per_step"]
        if dom in ("factor_compose", "factor_apply"):
            ach = flops / t_s / 1e12
            roofline = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_FP32_TFLOPS, "traffic": traffic,
                        "algorithmic_per_launch": flops / launches, "algorithmic_bytes_per_launch": byts / launches}
            if dom == "factor_compose":
                ex = alg["compose_executed"][0] / t_s / 1e12
                roofline.update({"executed_per_launch": alg["compose_executed"][0] / launches, "executed_achieved": ex,
                                 "executed_frac": ex / PEAK_FP32_TFLOPS})
        else:
            ach = byts / t_s / 1e9
            roofline = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "algorithmic_per_launch": byts / launches}
        for k in kernels:
            if k in alg and k != "compose_executed":
                t_k = kernels[k]["ms_per_step"] / 1e3
                kernels[k]["alg_tflops"] = alg[k][0] / t_k / 1e12
                kernels[k]["alg_gbs"] = alg[k][1] / t_k / 1e9

    # the per-pass measures of the paper's Table 5: N |Omega| / wall time of the factor epoch (N factor
    # passes with their C refreshes and shared-g passes) and of the core epoch, timed apart on extra steps
    f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t_f = t_c = 0.0
    for i in range(args.steps):
        f0.record()
        ft.factor_epoch(plan, prm, w.lr, w.lam)
        f1.record()
        ft.core_epoch(plan, prm, w.lr, w.lam)
        f2.record()
        torch.cuda.synchronize()
        t_f += f0.elapsed_time(f1) / args.steps
        t_c += f1.elapsed_time(f2) / args.steps
    passes = {"factor_ms": t_f, "core_ms": t_c, "factor_nnz_per_s": N * nnz / (t_f / 1e3),
              "core_nnz_per_s": N * nnz / (t_c / 1e3),
              "factor_core_nnz_updates_per_s": 2 * N * nnz / ((t_f + t_c) / 1e3),
              "note": "wall time of factor_epoch and core_epoch calls, timed apart after the measured steps"}

    cpu = None
    if not args.no_cpu_baseline:
        s = min(args.cpu_sample, nnz)
        log(f"CPU baseline: oracle on {s} elements")
        cpu = cpu_baseline(w, c, v, A, B, s)
        log(f"CPU baseline {cpu['value']:.3e} nnz-updates/s")

    line = {
        "metric": "SGD nnz updates/sec (factor+core)",
        "value": value,
        "unit": "nnz-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else "bf16 storage, f32 arithmetic",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {'x'.join(map(str, w.dims))}, {nnz} distinct coordinates, "
            f"Zipf({w.zipf}) per mode, values {w.value_kind}, J={J}, R={R}, lr={w.lr}, lam={w.lam}, init N(0,{w.sigma}^2)",
            "step": "factor pass + C refresh per mode, core pass + C refresh per mode, RMSE pass",
            "factor_passes": ("relaxed: chunks of long rows from the row at the start of the pass, guarded merge"
                              if args.relaxed else "exact serial SGD per row"),
            "fiber_shared_modes": [m for m in range(N) if fibers[m] is not None],
            "fibers_per_mode": [info["fibers"] for info in infos],
            "rmse_start": rmse0,
            "rmse_end": rmse,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "passes": passes,
        "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
