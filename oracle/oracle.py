"""FP64 CPU oracle for complex 2D Gaussian CGH -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It never imports the GPU package and the GPU package never
imports it; the two share nothing but the seeded input generators.

The heavy loops (rasterization, DFT, transfer function, adjoints) live in
``cgh_oracle.c``; this module marshals NumPy arrays and composes the steps in
the order of the paper's optimisation loop (Alg. 1): rasterize, zero-pad,
propagate, loss, and the adjoint chain.  The loss (Sec. 3.2, L_MSE), the
Adam update (Kingma & Ba, Algorithm 1, as configured for the 1080p workload)
and the finite-difference harness are plain NumPy.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

PARAM_KEYS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")
FLAG_PAPER_ALPHA = 2


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        f = ctypes.c_double
        u8 = ctypes.POINTER(ctypes.c_ubyte)
        L.orc_geometry.argtypes = [i, i, i, d, d, d, d, d]
        L.orc_raster_brute.argtypes = [i, i, i, i, f, i, d, d, d, d, d, d, d, d]
        L.orc_raster.argtypes = [i, i, i, i, f, i, d, d, d, d, d, d, d, d, d, d, d]
        L.orc_ambiguous_pixels.argtypes = [i, i, i, f, f, i, d, d, d, d, u8]
        L.orc_ambiguous_pixels.restype = ctypes.c_long
        L.orc_fft1.argtypes = [i, d, i]
        L.orc_fft2.argtypes = [i, i, d, i]
        L.orc_transfer.argtypes = [i, i, f, f, f, f, d]
        L.orc_propagate.argtypes = [i, i, i, i, i, f, d, i, d, f, d, d]
        L.orc_propagate_adjoint.argtypes = [i, i, i, i, i, f, d, i, d, f, d, d]
        L.orc_raster_adjoint.argtypes = [i, i, i, i, f, i, d, d, d, d, d, d, d, d, d, d, d, d, d]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Optics:
    """Problem geometry: canvas H x W, C channels, padded grid Hp x Wp,
    pixel pitch, one wavelength per channel, L propagation distances, support
    radius k (in standard deviations; k <= 0 means unbounded), and the optional
    circular aperture of Alg. 3 (radius in frequency bins of the padded grid,
    centred on the zero frequency; 0: none)."""

    def __init__(self, H, W, C, Hp, Wp, pitch, lambdas, zs, k=3.0, flags=0, aperture=0.0):
        self.H, self.W, self.C, self.Hp, self.Wp = int(H), int(W), int(C), int(Hp), int(Wp)
        self.pitch = float(pitch)
        self.lambdas = _f64(lambdas).reshape(-1)
        self.zs = _f64(zs).reshape(-1)
        self.k = float(k)
        self.flags = int(flags)
        self.aperture = float(aperture)
        assert self.lambdas.size == self.C

    @property
    def L(self):
        return self.zs.size


def widen(params):
    """FP32 parameter arrays -> exact FP64 copies (same keys)."""
    return {k: _f64(params[k]) for k in PARAM_KEYS}


def geometry(params, W, H):
    """Per-Gaussian activated quantities (Suppl. activations, covariance, inverse).
    Returns an [N, 12] array: mx, my, sx, sy, s00, s01, s11, det, i00, i01, i11, alpha."""
    p = widen(params)
    n = p["rotation"].shape[0]
    out = np.zeros((n, 12))
    lib().orc_geometry(n, W, H, _p(p["mean_pre"]), _p(p["log_scale"]), _p(p["rotation"]),
                       _p(p["opacity_pre"]), _p(out))
    return out


def raster(params, opt, brute=False, support=None):
    """Complex SLM field [C, H, W] = coherent sum of the Gaussians (Sec. 3.1).
    ``support``: optional parameter set whose geometry decides the k-sigma
    support predicate (holds the support fixed for finite differences)."""
    p = widen(params)
    n = p["rotation"].shape[0]
    C, H, W = opt.C, opt.H, opt.W
    re = np.zeros((C, H, W))
    im = np.zeros((C, H, W))
    if brute:
        assert support is None
        lib().orc_raster_brute(n, C, W, H, opt.k, opt.flags, _p(p["mean_pre"]),
                               _p(p["log_scale"]), _p(p["rotation"]), _p(p["amplitude"]),
                               _p(p["phase"]), _p(p["opacity_pre"]), _p(re), _p(im))
    else:
        s = widen(support) if support is not None else None
        null = ctypes.POINTER(ctypes.c_double)()
        lib().orc_raster(n, C, W, H, opt.k, opt.flags, _p(p["mean_pre"]), _p(p["log_scale"]),
                         _p(p["rotation"]), _p(p["amplitude"]), _p(p["phase"]),
                         _p(p["opacity_pre"]), _p(s["mean_pre"]) if s else null,
                         _p(s["log_scale"]) if s else null, _p(s["rotation"]) if s else null,
                         _p(re), _p(im))
    return re + 1j * im


def ambiguous_mask(params, opt, rel_band=1e-4):
    """Pixels touched by a (Gaussian, pixel) pair whose Mahalanobis distance lies
    within ``rel_band * k^2`` of the support boundary (or, with the Alg. 2
    weight, of its 1/255 skip boundary).  Returns (mask [H, W] bool, number of
    such pairs)."""
    p = widen(params)
    n = p["rotation"].shape[0]
    mask = np.zeros((opt.H, opt.W), dtype=np.uint8)
    cnt = lib().orc_ambiguous_pixels(n, opt.W, opt.H, opt.k, rel_band, opt.flags,
                                     _p(p["mean_pre"]),
                                     _p(p["log_scale"]), _p(p["rotation"]),
                                     _p(p["opacity_pre"]),
                                     mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    return mask.astype(bool), int(cnt)


def fft(x, inverse=False):
    """1-D DFT (own mixed-radix recursion); forward unnormalised, inverse 1/N."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().orc_fft1(a.shape[0], _p(a.view(np.float64)), int(inverse))
    return a


def fft2(x, inverse=False):
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().orc_fft2(a.shape[0], a.shape[1], _p(a.view(np.float64)), int(inverse))
    return a


def transfer(Hp, Wp, pitch, lam, z, aperture=0.0):
    """Band-limited angular-spectrum transfer function on the natural-order
    [Hp, Wp] frequency grid (Sec. 2; suppl. BLASM section)."""
    h = np.zeros((Hp, Wp), dtype=np.complex128)
    lib().orc_transfer(Hp, Wp, float(pitch), float(lam), float(z), float(aperture),
                       _p(h.view(np.float64)))
    return h


def propagate(field, opt):
    """[C, H, W] complex -> [L, C, H, W] complex: pad, FFT2, x H, IFFT2, crop."""
    f = np.ascontiguousarray(field, dtype=np.complex128)
    out = np.zeros((opt.L, opt.C, opt.H, opt.W), dtype=np.complex128)
    lib().orc_propagate(opt.C, opt.H, opt.W, opt.Hp, opt.Wp, opt.pitch, _p(opt.lambdas), opt.L,
                        _p(opt.zs), opt.aperture, _p(f.view(np.float64)),
                        _p(out.view(np.float64)))
    return out


def propagate_adjoint(grad_u, opt):
    """Adjoint of ``propagate``: conjugate transfer function, same band limit,
    summed over planes.  [L, C, H, W] -> [C, H, W]."""
    g = np.ascontiguousarray(grad_u, dtype=np.complex128)
    out = np.zeros((opt.C, opt.H, opt.W), dtype=np.complex128)
    lib().orc_propagate_adjoint(opt.C, opt.H, opt.W, opt.Hp, opt.Wp, opt.pitch,
                                _p(opt.lambdas), opt.L, _p(opt.zs), opt.aperture,
                                _p(g.view(np.float64)),
                                _p(out.view(np.float64)))
    return out


def mse(u, target):
    """L_MSE over all L*C*H*W intensities (Sec. 3.2), I = |u|^2.
    Returns (loss, intensity, grad_u) with grad_u = dL/dRe(u) + j dL/dIm(u)."""
    I = u.real ** 2 + u.imag ** 2
    T = np.asarray(target, dtype=np.float64).reshape(I.shape)
    M = I.size
    diff = I - T
    loss = float(np.sum(diff * diff) / M)
    dL_dI = 2.0 * diff / M
    grad_u = dL_dI * 2.0 * u
    return loss, I, grad_u


def recon(u, target, mask):
    """L_recon of Sec. 3.2 with each squared norm a mean over its elements (the
    reading taken for L_MSE): per plane ||I - T||^2 + ||I M - T M||^2 +
    ||I T - T T||^2, averaged over planes.  mask [L, H, W] is shared by the
    channels.  Returns (loss, intensity, grad_u), grad_u = dL/dRe(u) + j dL/dIm(u)."""
    I = u.real ** 2 + u.imag ** 2
    T = np.asarray(target, dtype=np.float64).reshape(I.shape)
    Mk = np.asarray(mask, dtype=np.float64).reshape(I.shape[0], 1, I.shape[2], I.shape[3])
    n = I.size
    r = I - T
    loss = float((np.sum(r * r) + np.sum((I * Mk - T * Mk) ** 2) + np.sum((I * T - T * T) ** 2))
                 / n)
    # d/dI of the three squared differences: 2 r (1 + M^2 + T^2)
    dL_dI = 2.0 * r * (1.0 + Mk * Mk + T * T) / n
    grad_u = dL_dI * 2.0 * u
    return loss, I, grad_u


# SSIM (Wang, Bovik, Sheikh and Simoncelli 2004, "Image quality assessment:
# from error visibility to structural similarity"), the L_SSIM term of the
# paper's final loss (Sec. 3.2).  Reading: 11 x 11 Gaussian window of standard
# deviation 1.5 normalised to sum 1, C1 = (0.01 R)^2 and C2 = (0.03 R)^2 with
# R = 1 (intensities in [0, 1]), windows fully inside the image.
SSIM_WIN = 11
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window():
    """1-D weights w_i (i = 0..10), exp(-(i - 5)^2 / (2 1.5^2)) normalised; the
    2-D window is w_i w_j."""
    i = np.arange(SSIM_WIN) - SSIM_WIN // 2
    w = np.exp(-(i * i) / (2.0 * 1.5 ** 2))
    return w / w.sum()


def _windows(a):
    """[H, W] -> [H - 10, W - 10, 11, 11]: the window at every valid position."""
    return np.lib.stride_tricks.sliding_window_view(a, (SSIM_WIN, SSIM_WIN))


def ssim_parts(x, y):
    """Window moments and SSIM at every valid position of two [H, W] images:
    mu_x, mu_y, sigma_x^2, sigma_y^2, sigma_xy (weighted by the window) and
    SSIM = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))."""
    w = ssim_window()
    w2 = np.outer(w, w)
    X, Y = _windows(np.asarray(x, np.float64)), _windows(np.asarray(y, np.float64))
    mx = np.einsum("abij,ij->ab", X, w2)
    my = np.einsum("abij,ij->ab", Y, w2)
    sxx = np.einsum("abij,ij->ab", X * X, w2) - mx * mx
    syy = np.einsum("abij,ij->ab", Y * Y, w2) - my * my
    sxy = np.einsum("abij,ij->ab", X * Y, w2) - mx * my
    n1, n2 = 2 * mx * my + SSIM_C1, 2 * sxy + SSIM_C2
    d1, d2 = mx * mx + my * my + SSIM_C1, sxx + syy + SSIM_C2
    return {"mu_x": mx, "mu_y": my, "s_xx": sxx, "s_yy": syy, "s_xy": sxy,
            "ssim": n1 * n2 / (d1 * d2), "n1": n1, "n2": n2, "d1": d1, "d2": d2}


def ssim_grad(x, y, coef):
    """d(sum_p coef(p) SSIM(p)) / dx for one image pair.  With the window sums
    mu_x = sum w x, e_xx = sum w x^2, e_xy = sum w x y, SSIM(p) depends on x(q)
    through w(q - p) [dS/dmu_x + 2 x(q) dS/de_xx + y(q) dS/de_xy], where
    dS/de_xx = dS/dsigma_x^2, dS/de_xy = dS/dsigma_xy and
    dS/dmu_x = (partial at fixed sigmas) - 2 mu_x dS/dsigma_x^2 - mu_y dS/dsigma_xy."""
    q = ssim_parts(x, y)
    S, mx, my = q["ssim"], q["mu_x"], q["mu_y"]
    den = q["d1"] * q["d2"]
    dS_dmx = 2 * my * q["n2"] / den - 2 * mx * S / q["d1"]
    dS_dsxx = -S / q["d2"]
    dS_dsxy = 2 * q["n1"] / den
    A = coef * (dS_dmx - 2 * mx * dS_dsxx - my * dS_dsxy)
    B = coef * dS_dsxx
    Cc = coef * dS_dsxy
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = ssim_window()
    g = np.zeros_like(x)
    Hv, Wv = S.shape
    for i in range(SSIM_WIN):
        for j in range(SSIM_WIN):
            xs, ys = x[i:i + Hv, j:j + Wv], y[i:i + Hv, j:j + Wv]
            g[i:i + Hv, j:j + Wv] += w[i] * w[j] * (A + 2 * xs * B + ys * Cc)
    return g


def ssim_loss(I, target):
    """L_SSIM = 1 - mean SSIM over every plane, channel and valid window
    position of I [L, C, H, W] against the target.  Returns (loss, dL/dI)."""
    I = np.asarray(I, np.float64)
    T = np.asarray(target, np.float64).reshape(I.shape)
    L, C, H, W = I.shape
    npos = L * C * (H - SSIM_WIN + 1) * (W - SSIM_WIN + 1)
    total = 0.0
    g = np.zeros_like(I)
    for l in range(L):
        for c in range(C):
            total += ssim_parts(I[l, c], T[l, c])["ssim"].sum()
            g[l, c] = -ssim_grad(I[l, c], T[l, c], 1.0 / npos)
    return 1.0 - total / npos, g


def full_loss(u, target, mask, ssim_weight):
    """The paper's final training loss (Sec. 3.2): L_recon (L_MSE without a
    mask) + ssim_weight L_SSIM.  Returns (loss, intensity, grad_u, psnr of the
    plain MSE)."""
    loss, I, grad_u = mse(u, target) if mask is None else recon(u, target, mask)
    ls, gI = ssim_loss(I, target)
    T = np.asarray(target, np.float64).reshape(I.shape)
    m = float(np.mean((I - T) ** 2))
    return loss + ssim_weight * ls, I, grad_u + ssim_weight * 2.0 * gI * u, 10.0 * np.log10(1.0 / m)


def raster_adjoint(params, grad_field, opt):
    """Gradients of the pre-activation parameters from dL/dU0 (suppl. Backward Pass)."""
    p = widen(params)
    n = p["rotation"].shape[0]
    C = opt.C
    g = np.ascontiguousarray(grad_field, dtype=np.complex128)
    out = {"mean_pre": np.zeros((n, 2)), "log_scale": np.zeros((n, 2)),
           "rotation": np.zeros(n), "amplitude": np.zeros((n, C)), "phase": np.zeros((n, C)),
           "opacity_pre": np.zeros(n)}
    lib().orc_raster_adjoint(n, C, opt.W, opt.H, opt.k, opt.flags, _p(p["mean_pre"]),
                             _p(p["log_scale"]), _p(p["rotation"]), _p(p["amplitude"]),
                             _p(p["phase"]), _p(p["opacity_pre"]), _p(g.view(np.float64)),
                             _p(out["mean_pre"]), _p(out["log_scale"]), _p(out["rotation"]),
                             _p(out["amplitude"]), _p(out["phase"]), _p(out["opacity_pre"]))
    return out


def forward(params, target, opt, support=None, mask=None, ssim_weight=0.0):
    """Alg. 1 forward: rasterize -> pad -> propagate -> |u|^2 -> L_MSE (or
    L_recon when a depth mask is given), plus ssim_weight L_SSIM if nonzero."""
    field = raster(params, opt, support=support)
    u = propagate(field, opt)
    out = {"field": field, "u": u}
    if ssim_weight:
        loss, I, grad_u, psnr = full_loss(u, target, mask, ssim_weight)
        out["psnr"] = psnr
    else:
        loss, I, grad_u = mse(u, target) if mask is None else recon(u, target, mask)
    out.update({"intensity": I, "loss": loss, "grad_u": grad_u})
    return out


def forward_backward(params, target, opt, mask=None, ssim_weight=0.0):
    """Forward plus the analytic adjoint chain; returns the forward dict with
    ``grad_field`` (dL/dU0) and ``grads`` (pre-activation parameter gradients)."""
    fwd = forward(params, target, opt, mask=mask, ssim_weight=ssim_weight)
    fwd["grad_field"] = propagate_adjoint(fwd["grad_u"], opt)
    fwd["grads"] = raster_adjoint(params, fwd["grad_field"], opt)
    return fwd


def loss_only(params, target, opt, support=None, mask=None):
    return forward(params, target, opt, support=support, mask=mask)["loss"]


def fd_gradient(params, target, opt, key, index, h=None, mask=None):
    """Central finite difference of the loss (L_MSE, or L_recon with a mask)
    w.r.t. one pre-activation parameter entry, in FP64, with the support held
    at the unperturbed parameters."""
    base = widen(params)
    flat = base[key].reshape(-1)
    x0 = float(flat[index])
    if h is None:
        h = 1e-6 * max(1.0, abs(x0))
    plus = {k: v.copy() for k, v in base.items()}
    minus = {k: v.copy() for k, v in base.items()}
    plus[key].reshape(-1)[index] = x0 + h
    minus[key].reshape(-1)[index] = x0 - h
    lp = loss_only(plus, target, opt, support=base, mask=mask)
    lm = loss_only(minus, target, opt, support=base, mask=mask)
    return (lp - lm) / (2.0 * h)


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Textbook Adam (Kingma & Ba 2015, Algorithm 1), FP64; returns new (p, m, v)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def adan(p, g, m, d, s, g_prev, t, lr, beta1=0.98, beta2=0.92, beta3=0.99, eps=1e-8,
         weight_decay=0.0):
    """Adan (Xie et al., Adan: Adaptive Nesterov Momentum Algorithm, Algorithm 1)
    with bias-corrected moments, decay-rate convention, FP64.  The gradient
    difference is taken as zero at the first step.  Returns (p, m, d, s, g)."""
    p, g, m, d, s, g_prev = (np.asarray(a, dtype=np.float64) for a in (p, g, m, d, s, g_prev))
    diff = np.zeros_like(g) if t == 1 else g - g_prev
    m = beta1 * m + (1.0 - beta1) * g
    d = beta2 * d + (1.0 - beta2) * diff
    nesterov = g + beta2 * diff
    s = beta3 * s + (1.0 - beta3) * nesterov * nesterov
    m_hat = m / (1.0 - beta1 ** t)
    d_hat = d / (1.0 - beta2 ** t)
    s_hat = s / (1.0 - beta3 ** t)
    p = p * (1.0 - lr * weight_decay) - lr * (m_hat + beta2 * d_hat) / (np.sqrt(s_hat) + eps)
    return p, m, d, s, g


def psnr(loss):
    """PSNR for intensities in [0, 1] from the mean squared error."""
    return 10.0 * np.log10(1.0 / loss)
