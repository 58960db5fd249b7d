#!/usr/bin/env python3
"""Throughput of the differentiable complex-Gaussian CGH step on one MI355X.

One step = cgh_rasterize (FP64 preprocess, binning, forward raster)
         + cgh_backward  (row FFT, column pass x H, row pass with |u|^2 / MSE /
                          adjoint seed, column pass x conj H, row IFFT, raster
                          adjoint, FP64 preprocess adjoint, loss reduction)
         + cgh_step      (Adam, lr 1e-3)
on the 1080p RGB workload: 1080 x 1920 SLM, 3 wavelengths (639, 515, 473 nm),
pitch 8 um, z = 5 mm, padded 2160 x 3840, 414,720 complex Gaussians (one per
5 pixels), seeded synthetic parameters and target.  Inputs are resident in HBM
before the timed region.  Prints one JSON line on stdout; diagnostics go to
stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# FP32 vector FMA issue rate without packed-FP32 instructions (this build never
# emits them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def in_support_pairs(p, H, W, k):
    """Exact number of (Gaussian, pixel) pairs with q <= k^2 (FP64, host)."""
    n = p["rotation"].shape[0]
    total = 0
    chunk = 8192
    for s in range(0, n, chunk):
        sl = slice(s, min(n, s + chunk))
        mx = 0.5 * (np.tanh(p["mean_pre"][sl, 0].astype(np.float64)) + 1) * W
        my = 0.5 * (np.tanh(p["mean_pre"][sl, 1].astype(np.float64)) + 1) * H
        sx = np.exp(p["log_scale"][sl, 0].astype(np.float64)) + 0.1
        sy = np.exp(p["log_scale"][sl, 1].astype(np.float64)) + 0.1
        th = p["rotation"][sl].astype(np.float64)
        c, si = np.cos(th), np.sin(th)
        s00 = sx * sx * c * c + sy * sy * si * si + 0.1
        s01 = (sx * sx - sy * sy) * c * si
        s11 = sx * sx * si * si + sy * sy * c * c + 0.1
        det = s00 * s11 - s01 * s01
        i00, i01, i11 = s11 / det, -s01 / det, s00 / det
        r = int(math.ceil(k * math.sqrt(max(s00.max(), s11.max())))) + 1
        off = np.arange(-r, r + 1, dtype=np.float64)
        px = np.floor(mx)[:, None, None] + off[None, None, :]
        py = np.floor(my)[:, None, None] + off[None, :, None]
        dx = px - mx[:, None, None]
        dy = py - my[:, None, None]
        q = i00[:, None, None] * dx * dx + 2 * i01[:, None, None] * dx * dy + i11[:, None, None] * dy * dy
        inside = (q <= k * k) & (px >= 0) & (px < W) & (py >= 0) & (py < H)
        total += int(inside.sum())
    return total


# kernel class -> source file holding its kernel (for matching committed counters)
KERNEL_SOURCE = {"col_pass": "fft_kernels.hip", "row_loss": "fft_kernels.hip",
                 "row_fft": "fft_kernels.hip", "raster": "raster_kernels.hip",
                 "raster_adjoint": "raster_kernels.hip"}


def measured_traffic(cls):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current source of that kernel; else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2511_15022_amd", "csrc", KERNEL_SOURCE.get(cls, ""))
    if not os.path.isfile(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*hbm_counters*.txt")):
        for line in open(path):
            parts = line.split()
            if len(parts) == 4 and parts[0] == "traffic" and parts[1] == cls and parts[3] == digest:
                return int(parts[2])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--workload", default="rgb_1080p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs the hot path on one GPU only; multi-GPU runs are not "
              "part of it (see the sharding note in DESIGN.md). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_15022_amd import binding, synth

    w = synth.WORKLOADS[args.workload]
    H, W, C, n = w["H"], w["W"], w["C"], w["n"]
    log(f"[bench] workload {args.workload}: {H}x{W} C={C} N={n} pad {w['Hp']}x{w['Wp']}")
    p = synth.params(w["pseed"], n, H, W, C)
    T_np = synth.target(w["tseed"], C, H, W)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    ctx = binding.Context(H, W, C, w["pitch"], w["lambdas"], w["zs"], pad=(w["Hp"], w["Wp"]),
                          max_gaussians=n, device=dev)
    P = binding.pack(p, device=dev)
    T = torch.from_numpy(T_np).to(dev)
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    gfield = torch.empty_like(field)
    G = torch.empty_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    loss = torch.zeros(2, dtype=torch.float64, device=dev)
    lr = 1e-3
    t_step = [0]

    def step():
        t_step[0] += 1
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=loss, grad_field=gfield, grads=G)
        binding.step(P, G, M, V, t_step[0], lr)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize(dev)
    pairs, ok = ctx.read_status()
    log(f"[bench] warmup done; tile pairs {pairs}; loss {loss[0].item():.6f} "
        f"psnr {loss[1].item():.3f} dB")

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize(dev)
    ms_total = start.elapsed_time(stop)
    ms_per_step = ms_total / args.steps
    pairs, ok = ctx.read_status()
    assert ok, "pair list overflow: timed steps incomplete"
    log(f"[bench] {args.steps} steps in {ms_total:.2f} ms -> {ms_per_step:.4f} ms/step; "
        f"loss {loss[0].item():.6f}")
    peak_vram = torch.cuda.max_memory_allocated(dev)
    if args.copy_probe:
        # a plain copy of known size: 256 MiB read + 256 MiB written per launch
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        log("[bench] copy probe: 3 x 268435456-byte device copies")
        del src, dst

    # per-kernel-class timing: HIP events around every launch of one class
    kernels = {}
    if not args.no_profile:
        for cls in binding.KERNEL_CLASSES:
            ctx.profile_begin(cls)
            for _ in range(args.profile_steps):
                step()
            ms, launches = ctx.profile_end()
            if launches:
                kernels[cls] = {"ms_per_step": ms / args.profile_steps,
                                "ms_per_launch": ms / launches,
                                "launches_per_step": launches / args.profile_steps}
        for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
            log(f"[bench]   {k:20s} {v['ms_per_step'] * 1e3:9.1f} us/step "
                f"({v['launches_per_step']:.0f} launches, {v['ms_per_launch'] * 1e3:.1f} us each)")

    # roofline of the dominant kernel class
    Hp, Wp = w["Hp"], w["Wp"]
    Hq, Wq = Hp // 2 + 1, Wp // 2 + 1
    hbm_bytes = {
        # read + write of the [C][H][Wp] buffer, plus the quarter transfer table
        "col_pass": 2 * C * H * Wp * 8 + C * Hq * Wq * 8,
        # read + write of the [C][H][Wp] buffer, plus the float target
        "row_loss": 2 * C * H * Wp * 8 + C * H * W * 4,
        # field [C][H][W] one way, [C][H][Wp] the other
        "row_fft": C * H * (W + Wp) * 8,
    }
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        t_launch = kernels[dom]["ms_per_launch"] * 1e-3
        if dom in hbm_bytes:
            achieved = hbm_bytes[dom] / t_launch / 1e9
            roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic(dom),
                        "algorithmic_bytes_per_launch": hbm_bytes[dom]}
        elif dom in ("raster", "raster_adjoint"):
            npairs = in_support_pairs(p, H, W, 3.0)
            per_pair = (10 + 4 * C) if dom == "raster" else (21 + 8 * C)
            achieved = npairs * per_pair / t_launch / 1e12
            roofline = {"kernel": dom, "bound": "alu", "achieved": achieved,
                        "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP32_VALU_PEAK_TFLOPS,
                        "traffic": measured_traffic(dom),
                        "in_support_pairs": npairs, "flop_per_pair": per_pair}
        else:
            roofline = {"kernel": dom, "bound": "unknown"}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        opt = O.Optics(H, W, C, Hp, Wp, w["pitch"], w["lambdas"], w["zs"])
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"[bench] oracle fwd+bwd on the host ({threads} threads)")
        reps = 0
        t0 = time.perf_counter()
        while reps < 1 or (time.perf_counter() - t0 < 10.0 and reps < 5):
            O.forward_backward(p, T_np, opt)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
        cpu = {"value": 1.0 / dt, "unit": "it/s", "cores": threads, "kind": "oracle",
               "sample": f"{reps} full fwd+bwd iteration(s) of the {args.workload} workload "
                         f"(raster, propagation, MSE, analytic adjoint; FP64), "
                         f"{dt:.2f} s each"}

    out = {
        "metric": "fwd+bwd iters/s, 1080p RGB 400k Gaussians",
        "value": 1000.0 / ms_per_step,
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "height": H, "width": W, "channels": C,
                   "gaussians": n, "pad": [Hp, Wp], "pitch_m": w["pitch"],
                   "wavelengths_m": w["lambdas"], "z_m": w["zs"], "step": "fwd+bwd+adam",
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_us_per_step": {k: round(v["ms_per_step"] * 1e3, 2) for k, v in kernels.items()},
        "tile_pairs": pairs,
        "peak_vram_gb": peak_vram / 1e9,
        "final_loss": loss[0].item(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
