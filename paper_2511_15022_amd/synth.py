"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws the
pre-activation parameters and target images that both the GPU library and the
CPU oracle then consume.  NumPy PCG64 streams, fully determined by the seed.

Parameters (shapes of the paper's primitive, Sec. 3.1; initial distributions
as configured for the benchmark workloads):
  mean_pre    [N, 2]  atanh(2 mu / [W, H] - 1) with mu ~ U[0, W) x U[0, H)
                      (the paper's position initialisation, Sec. 4)
  log_scale   [N, 2]  ~ N(ln 2, 0.3^2), per axis
  rotation    [N]     ~ U[0, pi)
  amplitude   [N, C]  ~ U[0, 1)
  phase       [N, C]  ~ U[0, 2 pi)
  opacity_pre [N]     = -0.5 (Sec. 4)
All stored as contiguous float32.

Targets: intensities in [0, 1], shaped like natural images: band-limited noise
plus painted disks and half-plane edges (recipe in ``target``).
"""
import math

import numpy as np

PARAM_KEYS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")


def params(seed, n, H, W, C, opacity_pre=-0.5, log_scale_mean=math.log(2.0),
           log_scale_std=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = np.empty((n, 2))
    mu[:, 0] = rng.uniform(0.0, W, n)
    mu[:, 1] = rng.uniform(0.0, H, n)
    u = 2.0 * mu / np.array([W, H], dtype=np.float64) - 1.0
    u = np.clip(u, -(1.0 - 1e-7), 1.0 - 1e-7)
    out = {
        "mean_pre": np.arctanh(u),
        "log_scale": rng.normal(log_scale_mean, log_scale_std, (n, 2)),
        "rotation": rng.uniform(0.0, math.pi, n),
        "amplitude": rng.uniform(0.0, 1.0, (n, C)),
        "phase": rng.uniform(0.0, 2.0 * math.pi, (n, C)),
        "opacity_pre": np.full(n, opacity_pre),
    }
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in out.items()}


def target(seed, C, H, W, L=1):
    """[L, C, H, W] float32 in [0, 1].  Per plane and channel:
    band-limited noise (white N(0, 1), keep radial |f| <= 1/32 cycles/px,
    min-max to [0, 1]); ceil(8 HW / 65536) disks of radius
    U[0.02, 0.15] min(H, W) and value U[0, 1] painted in order; four
    half-plane edges adding U[-0.3, 0.3]; T = clip(0.5 noise + 0.5 shapes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((L, C, H, W), dtype=np.float32)
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    keep = (fx * fx + fy * fy) <= (1.0 / 32.0) ** 2
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    n_disks = int(math.ceil(8.0 * H * W / 65536.0))
    for l in range(L):
        for c in range(C):
            white = rng.standard_normal((H, W))
            noise = np.real(np.fft.ifft2(np.fft.fft2(white) * keep))
            lo, hi = noise.min(), noise.max()
            noise = (noise - lo) / (hi - lo) if hi > lo else np.zeros_like(noise)
            shapes = np.zeros((H, W))
            for _ in range(n_disks):
                cx, cy = rng.uniform(0, W), rng.uniform(0, H)
                r = rng.uniform(0.02, 0.15) * min(H, W)
                val = rng.uniform(0.0, 1.0)
                # paint inside the disk's bounding box only (same pixels as a full test)
                y0, y1 = max(0, int(math.floor(cy - r))), min(H, int(math.ceil(cy + r)) + 1)
                x0, x1 = max(0, int(math.floor(cx - r))), min(W, int(math.ceil(cx + r)) + 1)
                sub = (xx[y0:y1, x0:x1] - cx) ** 2 + (yy[y0:y1, x0:x1] - cy) ** 2 <= r * r
                shapes[y0:y1, x0:x1][sub] = val
            for _ in range(4):
                ang = rng.uniform(0.0, 2.0 * math.pi)
                ox, oy = rng.uniform(0, W), rng.uniform(0, H)
                amt = rng.uniform(-0.3, 0.3)
                shapes += amt * (((xx - ox) * math.cos(ang) + (yy - oy) * math.sin(ang)) > 0)
            out[l, c] = np.clip(0.5 * noise + 0.5 * shapes, 0.0, 1.0)
    return out


def focal_masks(seed, L, H, W):
    """[L, H, W] float32 one-hot focal masks: a smooth random depth map
    (band-limited noise as in target(), radial |f| <= 1/64 cycles/px) split
    at its quantiles into L depth bins of equal area; mask l is 1 where the
    depth falls in bin l."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    keep = (fx * fx + fy * fy) <= (1.0 / 64.0) ** 2
    d = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((H, W))) * keep))
    edges = np.quantile(d, [l / L for l in range(1, L)])
    b = np.searchsorted(edges, d, side="right")
    return np.stack([(b == l) for l in range(L)]).astype(np.float32)


# Named workloads: (H, W, C, Hp, Wp, pitch_m, wavelengths_m, z_m, N, params seed, target seed);
# masks: per-depth targets trained with focal masks (the reconstruction loss)
WORKLOADS = {
    "tiny_256": dict(H=256, W=256, C=1, Hp=512, Wp=512, pitch=8e-6, lambdas=[515e-9],
                     zs=[2e-3], n=4096, pseed=0, tseed=1),
    "rgb_1080p": dict(H=1080, W=1920, C=3, Hp=2160, Wp=3840, pitch=8e-6,
                      lambdas=[639e-9, 515e-9, 473e-9], zs=[5e-3], n=414720, pseed=2, tseed=3),
    "bandlimit_stress": dict(H=256, W=256, C=1, Hp=512, Wp=512, pitch=8e-6, lambdas=[515e-9],
                             zs=[300e-3], n=4096, pseed=4, tseed=5),
    "rgb_4k": dict(H=2160, W=3840, C=3, Hp=4320, Wp=7680, pitch=3.74e-6,
                   lambdas=[639e-9, 515e-9, 473e-9], zs=[5e-3], n=1658880, pseed=6, tseed=7),
    "rgb_4k_3z": dict(H=2160, W=3840, C=3, Hp=4320, Wp=7680, pitch=3.74e-6,
                      lambdas=[639e-9, 515e-9, 473e-9], zs=[3e-3, 5e-3, 7e-3], n=1658880,
                      pseed=6, tseed=7, masks=True),
    # the shape of the paper's own measurements (Sec. 4): 3 x 640 x 1024, two
    # planes spanning the 4 mm volume around d0 = 3 mm, 532 nm green, pitch
    # 3.74 um, 65,536 Gaussians (the 5:1 parameter ratio)
    "paper_640x1024": dict(H=640, W=1024, C=3, Hp=1280, Wp=2048, pitch=3.74e-6,
                           lambdas=[639e-9, 532e-9, 473e-9], zs=[1e-3, 5e-3], n=65536,
                           pseed=8, tseed=9, masks=True),
}
