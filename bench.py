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
# FP32 vector FMA issue rate without packed-FP32 instructions (the library is
# compiled without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_description(threads):
    """CPU model, logical CPUs and the OpenMP thread setting of this host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"), "oracle_threads": threads}


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


def committed_figure(kind, cls, pattern):
    """A per-launch figure of kernel class ``cls`` from a committed rocprofv3
    summary under profiles/ (lines ``<kind> <class> <value> <sha256>``), if it
    was taken on the current source of that kernel; else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2511_15022_amd", "csrc", KERNEL_SOURCE.get(cls, ""))
    if not os.path.isfile(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", pattern)):
        for line in open(path):
            parts = line.split()
            if len(parts) == 4 and parts[0] == kind and parts[1] == cls and parts[3] == digest:
                return float(parts[2])
    return None


def measured_traffic(cls):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    v = committed_figure("traffic", cls, "*hbm_counters*.txt")
    return None if v is None else int(v)


VALU_CYCLES_PER_INST = 4     # a wave64 FP32 VALU instruction on a 16-lane SIMD
SIMDS, CLOCK_GHZ = 1024, 2.4  # MI355X: 256 CUs x 4 SIMDs


def profile_figures(cls, algorithmic, unit_scale, peak, t_launch_s):
    """Counter-based figures of a class: the kernel-trace duration and the
    fraction of peak it gives, the VALU floor from SQ_INSTS_VALU and the VALU
    issue utilisation against this run's own launch time."""
    out = {}
    dur = committed_figure("duration", cls, "*kernel_trace*.txt")
    if dur is not None:
        out["profile_duration_us"] = dur
        if algorithmic is not None:
            out["profile_frac"] = algorithmic / (dur * 1e-6) / unit_scale / peak
    insts = committed_figure("valu", cls, "*valu_counters*.txt")
    if insts is not None:
        floor_us = insts * VALU_CYCLES_PER_INST / SIMDS / (CLOCK_GHZ * 1e3)
        out["valu_insts_per_launch"] = insts
        out["valu_floor_us"] = floor_us
        out["valu_issue_util"] = floor_us / (t_launch_s * 1e6)
    return out


# ---------------------------------------------------------------------------
# Convergence from plain init: PSNR per optimiser step (logged on the device,
# no host sync inside the run) against wall-clock from HIP events.
# ---------------------------------------------------------------------------
def run_convergence(ctx, binding, p, T, n, steps, lr, dev, target_db=30.0):
    import numpy as np
    import torch
    P = binding.pack(p, device=dev)
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    G = torch.empty_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    log_t = torch.zeros((steps, 2), dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize(dev)
    ev[0].record()
    for i in range(steps):
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=log_t[i], grads=G)
        binding.step(P, G, M, V, i + 1, lr)
        ev[i + 1].record()
    torch.cuda.synchronize(dev)
    psnr = log_t[:, 1].cpu().numpy()  # PSNR of the parameters before update i
    t = np.array([ev[0].elapsed_time(ev[i + 1]) for i in range(steps)]) / 1e3
    hit = np.nonzero(psnr >= target_db)[0]
    best = int(np.argmax(psnr))
    marks = sorted({min(steps, m) for m in (1, 10, 50, 100, 200, 300, 400, 500)})
    return {
        "init": "plain (seeded random parameters of the workload)",
        "optimizer": f"Adam lr {lr:g} (0.9, 0.999, 1e-8)", "loss": "MSE",
        "steps": steps, "target_psnr_db": target_db,
        "seconds_to_target": float(t[hit[0]]) if len(hit) else None,
        "steps_to_target": int(hit[0]) + 1 if len(hit) else None,
        "best_psnr_db": float(psnr[best]), "seconds_to_best": float(t[best]),
        "psnr_db_at_step": {str(m): round(float(psnr[m - 1]), 3) for m in marks},
        "seconds_total": float(t[-1]),
    }


# The paper's optimisation recipe (Sec. 4): Adan with per-group learning
# rates, the position rate cosine-annealed from 1e-2 to 1e-3 over the run,
# scale 5e-3, rotation 1e-3, amplitude and phase 2.5e-3, opacity 2.5e-2, and
# the final loss L_MSE + 0.005 L_SSIM (one plane, so no focal masks).
PAPER_LR = {"mean_pre": (1e-2, 1e-3), "log_scale": 5e-3, "rotation": 1e-3,
            "amplitude": 2.5e-3, "phase": 2.5e-3, "opacity_pre": 2.5e-2}


def paper_lr_groups(i, steps):
    import math
    hi, lo = PAPER_LR["mean_pre"]
    pos = lo + 0.5 * (hi - lo) * (1.0 + math.cos(math.pi * i / max(steps - 1, 1)))
    return [pos] + [PAPER_LR[k] for k in ("log_scale", "rotation", "amplitude", "phase",
                                          "opacity_pre")]


def run_convergence_paper(binding, w, p, T, n, steps, dev, target_db=30.0, weight=0.005):
    import numpy as np
    import torch
    H, W, C = w["H"], w["W"], w["C"]
    # scales grow during a long run: room for 24 tiles per Gaussian on average
    ctx = binding.Context(H, W, C, w["pitch"], w["lambdas"], w["zs"], pad=(w["Hp"], w["Wp"]),
                          max_gaussians=n, max_pairs=24 * n + 65536, full_loss=True, device=dev)
    P = binding.pack(p, device=dev)
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    G = torch.empty_like(P)
    m, d, s, prev = (torch.zeros_like(P) for _ in range(4))
    log_t = torch.zeros((steps, 2), dtype=torch.float64, device=dev)
    groups = [paper_lr_groups(i, steps) for i in range(steps)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize(dev)
    ev[0].record()
    for i in range(steps):
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=log_t[i], grads=G, ssim_weight=weight)
        binding.step_adan(P, G, m, d, s, prev, i + 1, groups[i][0], lr_groups=groups[i],
                          channels=C)
        ev[i + 1].record()
    torch.cuda.synchronize(dev)
    _, ok = ctx.read_status(raise_on_overflow=False)
    psnr = log_t[:, 1].cpu().numpy()  # PSNR (plain MSE) of the parameters before update i
    t = np.array([ev[0].elapsed_time(ev[i + 1]) for i in range(steps)]) / 1e3
    hit = np.nonzero(psnr >= target_db)[0]
    best = int(np.argmax(psnr))
    marks = sorted({min(steps, k) for k in (1, 10, 100, 250, 500, 1000, 1500, 2000, 3000)})
    ctx.close()
    return {
        "init": "plain (seeded random parameters of the workload)",
        "optimizer": "Adan (0.98, 0.92, 0.99), per-group rates: position 1e-2 -> 1e-3 cosine, "
                     "scale 5e-3, rotation 1e-3, amplitude/phase 2.5e-3, opacity 2.5e-2",
        "loss": f"L_MSE + {weight:g} L_SSIM", "steps": steps, "target_psnr_db": target_db,
        "pair_capacity_ok": bool(ok),
        "seconds_to_target": float(t[hit[0]]) if len(hit) else None,
        "steps_to_target": int(hit[0]) + 1 if len(hit) else None,
        "best_psnr_db": float(psnr[best]), "seconds_to_best": float(t[best]),
        "psnr_db_at_step": {str(k): round(float(psnr[k - 1]), 3) for k in marks},
        "seconds_total": float(t[-1]),
    }


# Learned initialiser (the metric's "vs plain init" half): train the U-Net of
# paper_2511_15022_amd.learned_init end to end through this library on seeded
# 512 x 512 targets of the workload's geometry, move its weights to a network
# of the workload's size, and optimise from its prediction with the same Adam
# recipe as the plain-init run.  Seconds to the target PSNR count the
# network's inference (features, U-Net, lattice gather) plus the optimiser
# steps until the PSNR first reaches it.
def unet_flops(layers, H, W):
    f = 0
    for name, cu, cs, co, _ in layers:
        lev = 0 if name == "head" else int(name[3])
        f += 2 * (H >> lev) * (W >> lev) * 9 * (cu + cs) * co
    return f


def seconds_to(psnr, t, target_db, extra=0.0):
    """Seconds until the PSNR (of the parameters before each step) first
    reaches target_db: the steps before that one, plus ``extra``; None if never."""
    hit = np.nonzero(psnr >= target_db)[0]
    if not len(hit):
        return None, None
    t0 = np.concatenate([[0.0], t])
    return float(t0[hit[0]]) + extra, int(hit[0])


def summarise_starts(rows, target_db):
    """Median and worst case over targets of the seconds to target_db per start
    (a start that never reaches it counts as infinitely slow)."""
    out = {}
    for name in rows[0]["starts"]:
        secs = [r["starts"][name]["seconds_to_target"] for r in rows]
        best = [r["starts"][name]["best_psnr_db"] for r in rows]
        inf = [float("inf") if x is None else x for x in secs]
        med = float(np.median(inf))
        out[name] = {"reached": sum(x is not None for x in secs), "targets": len(rows),
                     "seconds_median": None if math.isinf(med) else med,
                     "seconds_worst": None if any(x is None for x in secs) else max(secs),
                     "best_psnr_db_median": float(np.median(best)),
                     "best_psnr_db_min": float(min(best))}
    return out


def run_learned_init(binding, w, T, n_plain, dev, train_steps, opt_steps, target_db=30.0,
                     lr_train=3e-4, lr=1e-3, train_size=512, pool=32, p_plain=None,
                     held_out=7):
    import numpy as np
    import torch
    from paper_2511_15022_amd import learned_init as LI, synth
    H, W, C = w["H"], w["W"], w["C"]
    z = w["zs"][0]
    ev = lambda: torch.cuda.Event(enable_timing=True)
    small = LI.Initializer(train_size, train_size, w["pitch"], w["lambdas"], z, seed=0, device=dev)
    LI.scale_head(small, 0.01)
    targets = [torch.from_numpy(synth.target(1000 + i, C, train_size, train_size)[0]).to(dev)
               for i in range(pool)]
    log, secs = LI.train(small, targets, train_steps, lr_train)
    big = LI.Initializer(H, W, w["pitch"], w["lambdas"], z, seed=0, device=dev)
    big.net.set_weights(small.net.get_weights())
    Tt = T.reshape(C, H, W)
    big.predict(Tt)  # warm-up
    a, b = ev(), ev()
    torch.cuda.synchronize(dev)
    a.record()
    learned = big.predict(Tt).clone()
    b.record()
    torch.cuda.synchronize(dev)
    infer = a.elapsed_time(b) / 1e3
    a2, b2 = ev(), ev()
    x = big.features(Tt)
    reps = 5  # back-to-back forwards, averaged
    a2.record()
    for _ in range(reps):
        big.net.forward(x)
    b2.record()
    torch.cuda.synchronize(dev)
    fwd = a2.elapsed_time(b2) / 1e3 / reps
    flops = unet_flops(big.net.layers, H, W)
    out = {"train": {"size": [train_size, train_size], "targets": pool, "steps": train_steps,
                     "seconds": secs, "ms_per_step": 1e3 * secs / train_steps, "lr": lr_train,
                     "psnr_db_first10": float(log[:10, 1].mean()),
                     "psnr_db_last20": float(log[-20:, 1].mean())},
           "network": {"params": big.net.n_params, "forward_ms": 1e3 * fwd,
                       "forward_tflops": flops / fwd / 1e12,
                       "mfma_bf16_peak_tflops": 2500.0,
                       "frac": flops / fwd / 1e12 / 2500.0},
           "gaussians": big.n, "inference_ms": 1e3 * infer, "target_psnr_db": target_db,
           "optimiser": f"Adam lr {lr:g} (0.9, 0.999, 1e-8)", "loss": "MSE"}
    for name, p0 in (("learned", learned), ("grid", big.grid())):
        psnr, t = LI.optimise(big.ctx, p0, big.n, Tt, opt_steps, lr)
        hit = np.nonzero(psnr >= target_db)[0]
        # PSNR i is that of the parameters before step i; reaching it at i
        # costs the i steps before it
        t0 = np.concatenate([[0.0], t])
        sec = None
        if len(hit):
            sec = float(t0[hit[0]]) + (infer if name == "learned" else 0.0)
        marks = sorted({min(opt_steps, k) for k in (1, 10, 50, 100, 200, 500)})
        out[name] = {"psnr_db_at_step": {str(k - 1): round(float(psnr[k - 1]), 3) for k in marks},
                     "best_psnr_db": float(psnr.max()), "seconds_to_target": sec,
                     "steps_to_target": int(hit[0]) if len(hit) else None}
    # held-out targets: the workload's own (seed 3) and `held_out` more of the
    # same recipe (seeds 2000 + i; the network trained on seeds 1000 .. 1031 at
    # 512 x 512), each optimised from the learned, grid and plain starts
    rows = []
    P_plain = binding.pack(p_plain, device=dev) if p_plain is not None else None
    for k, seed in enumerate([w["tseed"]] + [2000 + i for i in range(held_out)]):
        Tk = Tt if k == 0 else torch.from_numpy(synth.target(seed, C, H, W)[0]).to(dev)
        a, b = ev(), ev()
        a.record()
        pk = big.predict(Tk).clone()
        b.record()
        torch.cuda.synchronize(dev)
        inf_k = a.elapsed_time(b) / 1e3
        starts = {"learned": (pk, big.n, inf_k), "grid": (big.grid(), big.n, 0.0)}
        if P_plain is not None:
            starts["plain"] = (P_plain, n_plain, 0.0)
        row = {"target_seed": seed, "starts": {}}
        for name, (p0, nn, extra) in starts.items():
            psnr, t = LI.optimise(big.ctx, p0, nn, Tk, opt_steps, lr)
            sec, steps_to = seconds_to(psnr, t, target_db, extra)
            row["starts"][name] = {"seconds_to_target": sec, "steps_to_target": steps_to,
                                   "best_psnr_db": round(float(psnr.max()), 3),
                                   "psnr_db_at_step0": round(float(psnr[0]), 3)}
        rows.append(row)
    out["held_out"] = {"targets": len(rows), "steps": opt_steps,
                       "summary": summarise_starts(rows, target_db), "per_target": rows}
    pairs, ok = big.ctx.read_status(raise_on_overflow=False)
    out["pair_capacity_ok"] = bool(ok)
    out["_ctx"], out["_learned"] = big.ctx, learned  # for the POH leg; removed before printing
    out["_n"] = big.n
    return out


def psnr_of(u, T):
    """PSNR (dB) of |u|^2 against T, after the least-squares intensity scale
    (phase-only holograms have no amplitude freedom), on the host."""
    import numpy as np
    I = (u.real ** 2 + u.imag ** 2).double().cpu().numpy().reshape(-1)
    t = T.double().cpu().numpy().reshape(-1)
    s = float(I @ t / max(I @ I, 1e-300))
    return float(10 * np.log10(1.0 / np.mean((s * I - t) ** 2))), s


def run_poh(binding, ctx, params, n, T, steps, dev, opt_steps=200, lr=1e-3, lr_phase=0.1):
    """POH conversion (Sec. 3.3) at the workload's size: the Gaussians are first
    optimised from `params` (Adam, `opt_steps`); the Smooth POH is the
    double-phase coding of their field; the Random POH is optimised jointly
    with them under L_extract for `steps` steps from a seeded random phase."""
    import torch
    from paper_2511_15022_amd import learned_init as LI, poh
    C, H, W = ctx.C, ctx.H, ctx.W
    Tt = T.reshape(1, C, H, W)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # the complex hologram after the plain optimiser
    P = params.clone()
    field = torch.empty((C, H, W), dtype=torch.complex64, device=dev)
    G, M, V = torch.empty_like(P), torch.zeros_like(P), torch.zeros_like(P)
    for i in range(opt_steps):
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, Tt, grads=G)
        binding.step(P, G, M, V, i + 1, lr)
    ctx.rasterize(P, n, field)
    _, u = ctx.propagate(field, intensity=False, field_out=True)
    complex_db, _ = psnr_of(u, Tt)
    a, b = ev(), ev()
    torch.cuda.synchronize(dev)
    a.record()
    _, hs = poh.smooth(field)
    b.record()
    torch.cuda.synchronize(dev)
    # displayed through the circular aperture of Alg. 3 (half the Nyquist radius
    # of the longer padded side), which removes the double-phase carrier's
    # replica at the corner of the spectrum
    Hp, Wp = ctx.Hp, ctx.Wp
    apert = max(Hp, Wp) / 4.0
    actx = binding.Context(H, W, C, ctx.cfg.pitch_m, list(ctx.cfg.wavelength_m)[:C],
                           [ctx.cfg.z_m[0]], pad=(Hp, Wp), max_gaussians=1, aperture=apert,
                           device=dev)
    _, us = actx.propagate(hs, intensity=False, field_out=True)
    smooth_db, smooth_scale = psnr_of(us, Tt)
    _, us0 = ctx.propagate(hs, intensity=False, field_out=True)
    smooth_open_db, _ = psnr_of(us0, Tt)
    actx.close()
    rp = poh.RandomPOH(ctx, P, n, Tt, seed=7, lr_phase=lr_phase)
    a2, b2 = ev(), ev()
    torch.cuda.synchronize(dev)
    a2.record()
    for _ in range(steps):
        rp.step()
    b2.record()
    torch.cuda.synchronize(dev)
    u_g, u_r = rp.gradients()
    rand_db, rand_scale = psnr_of(u_r, Tt)
    return {"complex_hologram": {"optimiser_steps": opt_steps, "psnr_db": complex_db},
            "smooth_poh": {"method": "double-phase coding", "ms": a.elapsed_time(b),
                           "aperture_bins": apert, "psnr_db": smooth_db,
                           "intensity_scale": smooth_scale,
                           "psnr_db_without_aperture": smooth_open_db},
            "random_poh": {"steps": steps, "ms_per_step": a2.elapsed_time(b2) / steps,
                           "psnr_db": rand_db, "intensity_scale": rand_scale,
                           "gaussians_psnr_db": psnr_of(u_g, Tt)[0],
                           "loss": f"L_extract, l_comp 0.1, l_field 0.01, Adam lr {lr:g} "
                                   f"(Gaussians), {lr_phase:g} (phase)"},
            "psnr_note": "PSNR of the propagated intensity after the least-squares intensity scale"}


# ---------------------------------------------------------------------------
# Autodiff comparators: the same forward written with plain PyTorch ops and
# differentiated by torch.autograd, on the same GPU and inputs.
#   hybrid: this library's rasterizer and raster adjoint around an autodiff
#           BLASM (fft2, x H, ifft2, crop, |u|^2, MSE), the split the paper
#           compares against (its rasterizer stays native);
#   full:   the rasterization as well (a gather over the k-sigma boxes,
#           index_add into the canvas), then the same autodiff BLASM.
# Activations and the support test follow the paper's formulas (Sec. 3.1 and
# the supplementary rasterization equations); the grid is the same padded
# natural-order grid with the same FP32 transfer table.
# ---------------------------------------------------------------------------
def full_transfer(ctx, C, Hp, Wp, dev):
    import torch
    iy = torch.arange(Hp, device=dev)
    ix = torch.arange(Wp, device=dev)
    iy = torch.minimum(iy, Hp - iy)
    ix = torch.minimum(ix, Wp - ix)
    return torch.stack([ctx.get_transfer(c)[iy][:, ix] for c in range(C)])


def blasm_mse(field, Hf, T, H, W):
    import torch
    spec = torch.fft.fft2(field, s=tuple(Hf.shape[-2:]))  # zero-extends at the end
    u = torch.fft.ifft2(spec * Hf)[..., :H, :W]
    I = u.real * u.real + u.imag * u.imag
    return torch.mean((I - T) ** 2)


def raster_torch(binding, P, n, C, H, W, k=3.0):
    import torch
    v = binding.unpack(P, n, C)
    mp, ls, rot, amp, ph, op = (v[key] for key in binding.PARAM_KEYS)
    mx = 0.5 * (torch.tanh(mp[:, 0]) + 1.0) * W
    my = 0.5 * (torch.tanh(mp[:, 1]) + 1.0) * H
    sx = torch.exp(ls[:, 0]) + 0.1
    sy = torch.exp(ls[:, 1]) + 0.1
    c, s = torch.cos(rot), torch.sin(rot)
    s00 = sx * sx * c * c + sy * sy * s * s + 0.1
    s01 = (sx * sx - sy * sy) * c * s
    s11 = sx * sx * s * s + sy * sy * c * c + 0.1
    det = torch.clamp(s00 * s11 - s01 * s01, min=1e-10)
    i00, i01, i11 = s11 / det, -s01 / det, s00 / det
    alpha = torch.sigmoid(op)
    with torch.no_grad():  # pixels of each Gaussian's k-sigma box (indices only)
        rx, ry = k * torch.sqrt(s00), k * torch.sqrt(s11)
        x0 = torch.clamp(torch.ceil(mx - rx), min=0).long()
        x1 = torch.clamp(torch.floor(mx + rx), max=W - 1).long()
        y0 = torch.clamp(torch.ceil(my - ry), min=0).long()
        y1 = torch.clamp(torch.floor(my + ry), max=H - 1).long()
        nx = torch.clamp(x1 - x0 + 1, min=0)
        ny = torch.clamp(y1 - y0 + 1, min=0)
        cnt = nx * ny
        total = int(cnt.sum().item())
        g = torch.repeat_interleave(torch.arange(n, device=P.device), cnt, output_size=total)
        loc = torch.arange(total, device=P.device) - (torch.cumsum(cnt, 0) - cnt)[g]
        px = x0[g] + loc % nx[g]
        py = y0[g] + loc // nx[g]
        idx = py * W + px
    # pairs in chunks of 2^25: one gather of all 3e8 pairs of the 4K workload
    # loses gradient entries in PyTorch's backward
    fr = torch.zeros((C, H * W), dtype=P.dtype, device=P.device)
    fi = torch.zeros_like(fr)
    for s0 in range(0, total, 1 << 25):
        sl = slice(s0, min(total, s0 + (1 << 25)))
        gs = g[sl]
        dx = px[sl].to(P.dtype) - mx[gs]
        dy = py[sl].to(P.dtype) - my[gs]
        q = i00[gs] * dx * dx + 2.0 * i01[gs] * dx * dy + i11[gs] * dy * dy
        w = alpha[gs] * torch.where(q <= k * k, torch.exp(torch.clamp(-0.5 * q, min=-50.0)),
                                    torch.zeros_like(q))
        a = amp[gs] * w[:, None]
        fr = fr.index_add(1, idx[sl], (a * torch.cos(ph[gs])).t())
        fi = fi.index_add(1, idx[sl], (a * torch.sin(ph[gs])).t())
    return torch.complex(fr, fi).view(C, H, W), total


def run_autodiff(ctx, binding, P0, T, n, C, H, W, Hp, Wp, dev, reps=3):
    import torch
    Hf = full_transfer(ctx, C, Hp, Wp, dev)
    T0 = T[0]
    rest = torch.cuda.memory_allocated(dev)

    def timed(fn):
        fn()  # warm-up (plans, allocator)
        torch.cuda.synchronize(dev)
        torch.cuda.reset_peak_memory_stats(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize(dev)
        peak = torch.cuda.max_memory_allocated(dev)
        return out, e0.elapsed_time(e1) / reps, peak

    def fused():
        field = ctx.rasterize(P0, n)
        return ctx.backward(P0, n, field, T, grads=torch.empty_like(P0))

    def hybrid():
        f = ctx.rasterize(P0, n).detach().requires_grad_(True)
        blasm_mse(f, Hf, T0, H, W).backward()
        return ctx.rasterize_adjoint(P0, n, f.grad.contiguous())

    def full():
        Pg = P0.detach().clone().requires_grad_(True)
        field, _ = raster_torch(binding, Pg, n, C, H, W)
        blasm_mse(field, Hf, T0, H, W).backward()
        return Pg.grad

    def rel(a, b):
        va, vb = binding.unpack(a.detach(), n, C), binding.unpack(b.detach(), n, C)
        return max(float(torch.linalg.vector_norm(va[k] - vb[k]) /
                         torch.linalg.vector_norm(vb[k])) for k in binding.PARAM_KEYS)

    out = {"reps": reps, "resting_vram_gb": rest / 1e9,
           "what": "fwd+bwd of the MSE at the same parameters (no optimiser step)"}
    g_f, ms, peak = timed(fused)
    out["fused"] = {"ms": ms, "peak_vram_gb": peak / 1e9, "extra_vram_gb": (peak - rest) / 1e9}
    for name, fn in (("hybrid_autodiff_blasm", hybrid), ("full_autodiff", full)):
        try:
            g, ms, peak = timed(fn)
            out[name] = {"ms": ms, "peak_vram_gb": peak / 1e9,
                         "extra_vram_gb": (peak - rest) / 1e9,
                         "grad_rel_err_max_group": rel(g, g_f),
                         "fused_speedup": ms / out["fused"]["ms"]}
        except Exception as e:  # report, do not lose the headline line
            out[name] = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()
    return out


def run_serving(binding, dev, holograms, steps, seed=300, candidates=(1, 2)):
    """The serving batch: ``holograms`` seeded requests of sizes drawn from
    the five classes (512^2 .. 2048^2, one colour, n = pixels / 5, random
    wavelength of three and z in [2, 10] mm), each a ``steps``-step Adam solve.
    Served as batched solves: the requests of a size class run in one
    batched context, so each kernel of a step covers the whole class in one
    launch, captured as one HIP graph per batch.  The tile shape of each class
    comes from the project's autotuner (a short captured solve of the class
    batch at every shape), then the stream count from ``candidates`` (a
    warm-up run and a timed run each); the reported batch is the timed run of
    the best.  Then the per-hologram graphs of the single-hologram path on
    two streams, and a mixed run in which each class takes whichever of the
    two modes is faster per hologram and step (from the tile probe of its
    batch and its single solve), its class batches and single requests
    spread over two streams; the reported figures are those of the fastest
    of the three.  Beside them: the eager per-kernel calls on one stream."""
    import torch
    from paper_2511_15022_amd import serve
    reqs = serve.make_requests(holograms, seed=seed, device=dev)
    # the batched, single-hologram and mixed servers share two streams
    streams = [torch.cuda.Stream(device=dev) for _ in range(max(max(candidates), 2))]
    server = serve.BatchServer(steps, device=dev, streams=streams[:max(candidates)])
    best, rates, runs, tile_ms = serve.autotune_batched(server, reqs, candidates)
    for k, r in rates.items():
        log(f"[bench]   batched serving: {k} stream(s): {r:.2f} holograms/s")
    out = serve.summary(reqs, runs[best])
    classes = {}
    for r in reqs:
        classes.setdefault(f"{r.H}x{r.W}", 0)
        classes[f"{r.H}x{r.W}"] += 1
    batch_ms = {f"{h}x{w}x{b}": v for (h, w, b), v in server.batch_ms.items()}
    final_psnr = [float(r.out_loss[-1, 1].item()) for r in reqs]
    first_psnr = [float(r.out_loss[0, 1].item()) for r in reqs]
    tiles = {f"{h}x{w}": list(server.tile_of(h, w)) for (h, w) in tile_ms}
    # the single-hologram path: one graph per hologram, two streams
    for r in reqs:
        r.out_params = r.out_loss = None
    single = serve.Server(steps, device=dev, streams=streams[:2])
    costs = single.measure_class_costs(reqs)
    single.run(reqs, streams=2)
    res2 = single.run(reqs, streams=2)
    per_holo = len(reqs) / res2["wall_s"]
    # the mixed path: each class in its faster mode (per hologram and step,
    # from the tile probe of its batch and its single solve), two streams
    probe_steps = 20
    first_batch = {}
    for bt in serve.batches_of(reqs, server.max_batch):
        first_batch.setdefault((bt[0].H, bt[0].W), len(bt))
    batch_step_ms = {key: (tile_ms[key][server.tile_of(*key)] / probe_steps, first_batch[key])
                     for key in tile_ms}
    single_step_ms = {key: v / steps for key, v in costs.items()}
    mixed = serve.MixedServer(server, single, batch_step_ms, single_step_ms)
    if server.streams[:2] != single.streams:
        raise RuntimeError("serving servers must share their streams")
    for r in reqs:
        r.out_params = r.out_loss = None
    mixed.run(reqs, streams=2)
    res3 = mixed.run(reqs, streams=2)
    mixed_rate = len(reqs) / res3["wall_s"]
    mixed_classes = sorted(f"{h}x{w}" for (h, w) in mixed.batched)
    del mixed, server
    torch.cuda.empty_cache()
    # eager comparator: the same solves, one host call per kernel group, one stream
    ctxs = {key: single.slot(0, *key, key[0] * key[1] // 5).ctx for key in costs}
    bufs = {key: torch.empty_like(next(r.params for r in reqs if (r.H, r.W) == key))
            for key in costs}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        ctx = ctxs[(r.H, r.W)]
        P = bufs[(r.H, r.W)]
        P.copy_(r.params)
        ctx.set_optics([r.wavelength], [r.z])
        serve.solve_eager(ctx, P, r.n, r.target, steps)
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    # the reported mode is the fastest of the three, each measured the same
    # way (a warm-up run, then the timed run)
    batched_rate = out["holograms_per_s"]
    modes = {"batched": (batched_rate, best, None),
             "single": (per_holo, 2, serve.summary(reqs, res2)),
             "mixed": (mixed_rate, 2, serve.summary(reqs, res3))}
    pick = max(modes, key=lambda k: modes[k][0])
    if modes[pick][2] is not None:
        out.update(modes[pick][2])
    describe = {
        "batched": "batched contexts: one launch per kernel per class batch, one graph per batch",
        "single": "single-hologram contexts: one graph per hologram, two streams",
        "mixed": "mixed: each class batched or one hologram at a time, whichever is faster "
                 "per hologram, the jobs on two streams"}
    out.update({
        "steps_per_solve": steps,
        "mode": describe[pick],
        "holograms_per_s_by_mode": {k: v[0] for k, v in modes.items()},
        "mixed_batched_classes": mixed_classes,
        "streams": modes[pick][1],
        "batched_streams": best,
        "autotune_holograms_per_s": {str(k): v for k, v in rates.items()},
        "tile_per_class": tiles,
        "tile_autotune_ms": {f"{h}x{w}": {f"{a}x{b}": round(v, 3) for (a, b), v in t.items()}
                             for (h, w), t in tile_ms.items()},
        "class_counts": classes,
        "batch_solve_ms": batch_ms,
        "single_hologram_graphs_two_streams_holograms_per_s": per_holo,
        "single_hologram_class_step_us": {f"{h}x{w}": 1e3 * v / steps
                                          for (h, w), v in costs.items()},
        "eager_one_stream_holograms_per_s": len(reqs) / eager_s,
        "batched_speedup_vs_single_graphs": batched_rate / per_holo,
        "psnr_db_first_step_median": float(np.median(first_psnr)),
        "psnr_db_last_step_median": float(np.median(final_psnr)),
        "data": "synthetic, seeded (serve.make_requests, seed 300)",
    })
    del single, reqs
    return out


# The paper's own figures for its workload (Sec. 4 and Table 3, one NVIDIA
# RTX 3090): 2000 steps in 1.4 min (about 42 ms per step, with L_recon +
# SSIM, Adan and Python overhead), 2.2 GB of VRAM, and 2.13 ms to render
# (rasterize + propagate) at the 5:1 ratio.
PAPER_FIGURES = {"hardware": "NVIDIA RTX 3090", "ms_per_step": 42.0, "vram_gb": 2.2,
                 "render_ms": 2.13, "workload": "3 x 1024 x 640, L = 2, 5:1 ratio (65,536 "
                 "Gaussians), first 50 DIV2K images", "source": "Sec. 4 results and Table 3"}


def run_paper_context(binding, dev, steps, weight=0.005):
    """The paper-shaped workload (synth.WORKLOADS['paper_640x1024']) with the
    paper's recipe: L_recon with focal masks + 0.005 L_SSIM, Adan with the
    per-group rates; ms per step, the forward-only render time (rasterize +
    propagate to both planes' intensities) and the peak VRAM of the leg,
    beside the paper's figures on its own hardware."""
    import torch
    from paper_2511_15022_amd import synth
    w = synth.WORKLOADS["paper_640x1024"]
    H, W, C, n, L = w["H"], w["W"], w["C"], w["n"], len(w["zs"])
    torch.cuda.synchronize(dev)
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    p = synth.params(w["pseed"], n, H, W, C)
    T = torch.from_numpy(synth.target(w["tseed"], C, H, W, L=L)).to(dev)
    Mk = torch.from_numpy(synth.focal_masks(w["tseed"] + 1, L, H, W)).to(dev)
    ctx = binding.Context(H, W, C, w["pitch"], w["lambdas"], w["zs"], pad=(w["Hp"], w["Wp"]),
                          max_gaussians=n, full_loss=True, device=dev)
    P = binding.pack(p, device=dev)
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    G = torch.empty_like(P)
    m, d, s, prev = (torch.zeros_like(P) for _ in range(4))
    loss = torch.zeros(2, dtype=torch.float64, device=dev)
    t = [0]

    def step():
        t[0] += 1
        g = paper_lr_groups(t[0] - 1, 2000)
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=loss, grads=G, mask=Mk, ssim_weight=weight)
        binding.step_adan(P, G, m, d, s, prev, t[0], g[0], lr_groups=g, channels=C)

    for _ in range(3):
        step()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize(dev)
    ms = a.elapsed_time(b) / steps
    # render: rasterize + propagate (intensity of both planes)
    I = torch.empty(ctx.plane_shape(), dtype=torch.float32, device=dev)

    def render():
        ctx.rasterize(P, n, field)
        binding.lib().cgh_propagate(ctx.handle, binding._ptr(field), binding._ptr(I), None,
                                    binding._stream(dev))

    for _ in range(3):
        render()
    torch.cuda.synchronize(dev)
    a.record()
    for _ in range(steps):
        render()
    b.record()
    torch.cuda.synchronize(dev)
    render_ms = a.elapsed_time(b) / steps
    _, ok = ctx.read_status()
    peak = torch.cuda.max_memory_allocated(dev) - base
    out = {"workload": "paper_640x1024", "height": H, "width": W, "channels": C, "planes": L,
           "z_m": w["zs"], "gaussians": n, "pitch_m": w["pitch"], "wavelengths_m": w["lambdas"],
           "loss": f"L_recon with focal masks + {weight:g} L_SSIM",
           "optimizer": "Adan, per-group rates", "ms_per_step": ms, "it_per_s": 1e3 / ms,
           "render_ms": render_ms, "peak_vram_gb": peak / 1e9,
           "workspace_gb": ctx.workspace_bytes / 1e9, "paper": PAPER_FIGURES,
           "step_speedup_vs_paper": PAPER_FIGURES["ms_per_step"] / ms,
           "render_speedup_vs_paper": PAPER_FIGURES["render_ms"] / render_ms}
    ctx.close()
    return out


def run_paper_loss(binding, w, p, T, Mk, n, steps, dev, weight=0.005):
    """The same step with the paper's final loss, L_recon (L_MSE without masks)
    + weight L_SSIM, on a context that holds the SSIM workspace; times `steps`
    steps after 3 warmup steps, and the SSIM kernels (loss class) alone."""
    import torch
    H, W, C = w["H"], w["W"], w["C"]
    ctx = binding.Context(H, W, C, w["pitch"], w["lambdas"], w["zs"], pad=(w["Hp"], w["Wp"]),
                          max_gaussians=n, full_loss=True, device=dev)
    P = binding.pack(p, device=dev)
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
    G = torch.empty_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    loss = torch.zeros(2, dtype=torch.float64, device=dev)
    t = [0]

    def step():
        t[0] += 1
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=loss, grads=G, mask=Mk, ssim_weight=weight)
        binding.step(P, G, M, V, t[0], 1e-3)

    for _ in range(3):
        step()
    torch.cuda.synchronize(dev)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize(dev)
    ms = a.elapsed_time(b) / steps
    ctx.profile_begin("loss")
    for _ in range(3):
        step()
    ms_loss, _ = ctx.profile_end()
    out = {"ms_per_step": ms, "value": 1000.0 / ms, "unit": "it/s", "steps": steps,
           "ssim_weight": weight, "loss": "L_recon + 0.005 L_SSIM" if Mk is not None
           else "L_MSE + 0.005 L_SSIM", "final_loss": loss[0].item(),
           "psnr_db": loss[1].item(), "ssim_us_per_step": ms_loss / 3 * 1e3,
           "workspace_bytes": ctx.workspace_bytes}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--workload", default="rgb_1080p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--convergence-steps", type=int, default=500,
                    help="optimiser steps of the PSNR-vs-time run from plain init (0: skip)")
    ap.add_argument("--no-autodiff", action="store_true",
                    help="skip the fused-vs-autodiff comparison")
    ap.add_argument("--paper-convergence-steps", type=int, default=2000,
                    help="steps of the run with the paper's optimiser recipe and final loss "
                         "from plain init (0: skip)")
    ap.add_argument("--poh-steps", type=int, default=200,
                    help="Random POH steps after the learned initialiser leg (0: skip)")
    ap.add_argument("--learned-init-steps", type=int, default=600,
                    help="training steps of the learned initialiser (0: skip)")
    ap.add_argument("--held-out-targets", type=int, default=7,
                    help="further 1080p targets the learned, grid and plain starts are "
                         "optimised on (beside the workload's own)")
    ap.add_argument("--paper-context-steps", type=int, default=20,
                    help="timed steps of the paper-shaped workload (0: skip)")
    ap.add_argument("--paper-loss-steps", type=int, default=20,
                    help="timed steps with the paper's final loss, L + 0.005 L_SSIM (0: skip)")
    ap.add_argument("--serving-holograms", type=int, default=64,
                    help="holograms in the serving batch (0: skip)")
    ap.add_argument("--serving-steps", type=int, default=300,
                    help="Adam steps per hologram solve in the serving batch")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the hot path runs on one GPU; runs over several GPUs are not "
              "implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_15022_amd import binding, synth

    w = synth.WORKLOADS[args.workload]
    H, W, C, n = w["H"], w["W"], w["C"], w["n"]
    log(f"[bench] workload {args.workload}: {H}x{W} C={C} N={n} pad {w['Hp']}x{w['Wp']}")
    p = synth.params(w["pseed"], n, H, W, C)
    L = len(w["zs"])
    T_np = synth.target(w["tseed"], C, H, W, L=L)
    Mk_np = synth.focal_masks(w["tseed"] + 1, L, H, W) if w.get("masks") else None
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    torch.cuda.reset_peak_memory_stats(dev)
    ctx = binding.Context(H, W, C, w["pitch"], w["lambdas"], w["zs"], pad=(w["Hp"], w["Wp"]),
                          max_gaussians=n, device=dev)
    P = binding.pack(p, device=dev)
    T = torch.from_numpy(T_np).to(dev)
    Mk = torch.from_numpy(Mk_np).to(dev) if Mk_np is not None else None
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
        if Mk is None:
            # the L_MSE backward with the Adam update fused into its last kernel
            ctx.backward_step(P, n, field, T, M, V, t_step[0], lr, loss=loss,
                              grad_field=gfield)
        else:
            ctx.backward(P, n, field, T, loss=loss, grad_field=gfield, grads=G, mask=Mk)
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
    # the same steps as one HIP-graph launch (cgh_solve: rasterize, backward and
    # Adam per step, captured once; L_MSE only, so not for the masked workloads)
    ms_per_step_eager, graph = ms_per_step, None
    if Mk is None and args.steps > 0:
        Pg = binding.pack(p, device=dev)
        sol = binding.Solve(ctx, Pg, n, T, args.steps, lr=lr)
        sol.launch()  # warm-up launch
        torch.cuda.synchronize(dev)
        Pg.copy_(P)
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(sol.stream)
        sol.launch()
        g1.record(sol.stream)
        torch.cuda.synchronize(dev)
        ms_graph = g0.elapsed_time(g1) / args.steps
        pairs_g, ok_g = ctx.read_status()
        assert ok_g, "pair list overflow in the graph-launched steps"
        graph = {"ms_per_step": ms_graph, "steps": args.steps,
                 "final_loss": sol.loss_log[-1, 0].item(),
                 "what": "the timed steps as one cgh_solve graph launch (moments zeroed at its "
                         "start), from the parameters the eager steps ended with"}
        sol.close()
        del Pg, sol
        log(f"[bench] graph-launched: {args.steps} steps -> {ms_graph:.4f} ms/step "
            f"(eager calls {ms_per_step_eager:.4f} ms/step)")
        ms_per_step = min(ms_per_step, ms_graph)
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
    # per-pair and per-Gaussian byte counts of the record layouts (C channels)
    rec_stride = (((9 + 2 * C) + 3) & ~3) + 4
    part_stride = ((2 * C + 5) + 3) & ~3
    nparam = 6 + 2 * C
    hbm_bytes["preprocess"] = n * (nparam * 4 + rec_stride * 4 + 8 + 4)
    hbm_bytes["preprocess_adjoint"] = n * (2 * nparam * 4 + 8) + pairs * part_stride * 4
    npairs_cache = []

    def class_roofline(cls):
        t_launch = kernels[cls]["ms_per_launch"] * 1e-3
        if cls in hbm_bytes:
            achieved = hbm_bytes[cls] / t_launch / 1e9
            r = {"kernel": cls, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                 "traffic": measured_traffic(cls),
                 "algorithmic_bytes_per_launch": hbm_bytes[cls]}
            r.update(profile_figures(cls, hbm_bytes[cls], 1e9, HBM_PEAK_GBS, t_launch))
            return r
        if cls in ("raster", "raster_adjoint"):
            if not npairs_cache:
                npairs_cache.append(in_support_pairs(p, H, W, 3.0))
            npairs = npairs_cache[0]
            per_pair = (10 + 4 * C) if cls == "raster" else (21 + 8 * C)
            achieved = npairs * per_pair / t_launch / 1e12
            r = {"kernel": cls, "bound": "alu", "achieved": achieved,
                 "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": measured_traffic(cls),
                 "in_support_pairs": npairs, "flop_per_pair": per_pair}
            r.update(profile_figures(cls, npairs * per_pair, 1e12, FP32_VALU_PEAK_TFLOPS,
                                     t_launch))
            return r
        label = {"binning": "latency (integer sort, five short launches)",
                 "loss": "latency (one-block FP64 reduction)"}.get(cls, "latency")
        return {"kernel": cls, "bound": label}

    roofline = None
    rooflines = {}
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        roofline = class_roofline(dom)
        for cls in kernels:
            r = class_roofline(cls)
            rooflines[cls] = {k: r[k] for k in ("bound", "achieved", "unit", "frac",
                                                "profile_frac", "valu_floor_us",
                                                "valu_issue_util") if k in r}

    paper_loss = None
    if args.paper_loss_steps > 0:
        log(f"[bench] paper's final loss (+ 0.005 L_SSIM): {args.paper_loss_steps} steps")
        try:
            paper_loss = run_paper_loss(binding, w, p, T, Mk, n, args.paper_loss_steps, dev)
            log(f"[bench]   {paper_loss['ms_per_step']:.4f} ms/step; "
                f"ssim kernels {paper_loss['ssim_us_per_step']:.1f} us/step")
        except Exception as e:
            paper_loss = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()

    conv = None
    if args.convergence_steps > 0 and L == 1 and Mk is None:
        log(f"[bench] convergence from plain init: {args.convergence_steps} Adam steps")
        try:
            conv = run_convergence(ctx, binding, p, T, n, args.convergence_steps, lr, dev)
            log(f"[bench]   best PSNR {conv['best_psnr_db']:.2f} dB at "
                f"{conv['seconds_to_best']:.3f} s; 30 dB at {conv['seconds_to_target']} s")
        except Exception as e:
            conv = {"error": f"{type(e).__name__}: {e}"[:300]}
    conv_paper = None
    if args.paper_convergence_steps > 0 and L == 1 and Mk is None:
        log(f"[bench] convergence with the paper's recipe: {args.paper_convergence_steps} "
            f"Adan steps, L_MSE + 0.005 L_SSIM")
        try:
            conv_paper = run_convergence_paper(binding, w, p, T, n,
                                               args.paper_convergence_steps, dev)
            log(f"[bench]   best PSNR {conv_paper['best_psnr_db']:.2f} dB at "
                f"{conv_paper['seconds_to_best']:.3f} s; 30 dB at "
                f"{conv_paper['seconds_to_target']} s; {conv_paper['psnr_db_at_step']}")
        except Exception as e:
            conv_paper = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()
    learned = None
    if args.learned_init_steps > 0 and L == 1 and Mk is None:
        log(f"[bench] learned initialiser: {args.learned_init_steps} training steps at 512 x 512")
        try:
            learned = run_learned_init(binding, w, T, n, dev, args.learned_init_steps,
                                       max(args.convergence_steps, 200), p_plain=p,
                                       held_out=args.held_out_targets)
            log(f"[bench]   train {learned['train']['seconds']:.2f} s "
                f"({learned['train']['ms_per_step']:.2f} ms/step); inference "
                f"{learned['inference_ms']:.2f} ms; U-Net forward "
                f"{learned['network']['forward_ms']:.2f} ms "
                f"({learned['network']['forward_tflops']:.1f} TFLOP/s)")
            for k in ("learned", "grid"):
                log(f"[bench]   {k}: {learned[k]}")
            log(f"[bench]   held-out targets: {learned['held_out']['summary']}")
            if args.poh_steps > 0:
                log(f"[bench] POH conversion: {args.poh_steps} Random POH steps")
                try:
                    learned["poh"] = run_poh(binding, learned["_ctx"], learned["_learned"],
                                             learned["_n"], T, args.poh_steps, dev)
                    log(f"[bench]   {learned['poh']}")
                except Exception as e:
                    learned["poh"] = {"error": f"{type(e).__name__}: {e}"[:300]}
        except Exception as e:
            learned = {"error": f"{type(e).__name__}: {e}"[:300]}
        if isinstance(learned, dict):
            for k in ("_ctx", "_learned", "_n"):
                learned.pop(k, None)
        torch.cuda.empty_cache()
    autodiff = None
    if not args.no_autodiff and L == 1 and Mk is None:
        log("[bench] fused adjoint vs autodiff (same GPU, same inputs)")
        try:
            P0 = binding.pack(p, device=dev)
            autodiff = run_autodiff(ctx, binding, P0, T, n, C, H, W, w["Hp"], w["Wp"], dev)
            for k, v in autodiff.items():
                if isinstance(v, dict):
                    log(f"[bench]   {k}: {v}")
            del P0
        except Exception as e:
            autodiff = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()

    paper_ctx = None
    if args.paper_context_steps > 0 and args.workload == "rgb_1080p":
        log(f"[bench] paper-shaped workload: {args.paper_context_steps} steps")
        try:
            paper_ctx = run_paper_context(binding, dev, args.paper_context_steps)
            log(f"[bench]   {paper_ctx['ms_per_step']:.3f} ms/step, render "
                f"{paper_ctx['render_ms']:.3f} ms, peak {paper_ctx['peak_vram_gb']:.2f} GB "
                f"(paper on an RTX 3090: 42 ms, 2.13 ms, 2.2 GB)")
        except Exception as e:
            paper_ctx = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()

    serving = None
    if args.serving_holograms > 0 and args.workload == "rgb_1080p":
        log(f"[bench] serving batch: {args.serving_holograms} holograms x "
            f"{args.serving_steps} steps")
        try:
            serving = run_serving(binding, dev, args.serving_holograms, args.serving_steps)
            log(f"[bench]   by mode: " + ", ".join(
                f"{k} {v:.2f}" for k, v in serving['holograms_per_s_by_mode'].items())
                + f" holograms/s (mixed batches {serving['mixed_batched_classes']})")
            log(f"[bench]   {serving['holograms_per_s']:.2f} holograms/s ({serving['mode']}); "
                f"latency p50 {serving['latency_p50_ms']:.1f} ms "
                f"p99 {serving['latency_p99_ms']:.1f} ms; eager "
                f"{serving['eager_one_stream_holograms_per_s']:.2f} holograms/s")
        except Exception as e:
            serving = {"error": f"{type(e).__name__}: {e}"[:300]}
        torch.cuda.empty_cache()

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
                         f"{dt:.2f} s each",
               "host": host_description(threads)}

    out = {
        "metric": ("fwd+bwd iters/s, 1080p RGB 400k Gaussians; seconds to 30 dB vs plain init"
                   if args.workload == "rgb_1080p" else f"fwd+bwd iters/s, {args.workload}"),
        "value": 1000.0 / ms_per_step,
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_eager_calls": ms_per_step_eager,
        "graph_launched": graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "height": H, "width": W, "channels": C,
                   "gaussians": n, "pad": [Hp, Wp], "pitch_m": w["pitch"],
                   "wavelengths_m": w["lambdas"], "z_m": w["zs"], "step": "fwd+bwd+adam",
                   "loss": "L_recon with focal masks" if Mk is not None else "MSE",
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "rooflines": rooflines,
        "cpu_baseline": cpu,
        "convergence": conv,
        "convergence_paper_recipe": conv_paper,
        "learned_init": learned,
        "autodiff": autodiff,
        "paper_loss": paper_loss,
        "serving_batch": serving,
        "paper_context": paper_ctx,
        "kernels_us_per_step": {k: round(v["ms_per_step"] * 1e3, 2) for k, v in kernels.items()},
        "tile_pairs": pairs,
        "peak_vram_gb": peak_vram / 1e9,
        "final_loss": loss[0].item(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
