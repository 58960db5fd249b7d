"""Pins the oracle's hand-derived adjoint (supplementary Backward Pass, chained
through the activations of Sec. 3.1) to automatic differentiation: the forward
is restated here from the paper's formulas with torch operations in FP64
(brute force over every pixel and Gaussian, FFT-based propagation with the
band-limited transfer function, L_MSE or L_recon, optionally + L_SSIM), and
torch.autograd differentiates it.  The support indicator q <= k^2 is piecewise constant, so
both sides differentiate the same function; agreement is to rounding."""
import numpy as np
import pytest
import torch

from paper_2511_15022_amd import synth

KEYS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")


def torch_ssim(I, T):
    """1 - mean SSIM (11 x 11 Gaussian window, sigma 1.5; C1 = 0.01^2,
    C2 = 0.03^2; windows inside the image) with separable conv2d filtering."""
    i = torch.arange(11, dtype=torch.float64) - 5
    w = torch.exp(-(i * i) / (2 * 1.5 ** 2))
    w = w / w.sum()
    L, C, H, W = I.shape
    x, y = I.reshape(L * C, 1, H, W), T.reshape(L * C, 1, H, W)

    def f(a):
        a = torch.nn.functional.conv2d(a, w.view(1, 1, 1, 11))
        return torch.nn.functional.conv2d(a, w.view(1, 1, 11, 1))

    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    s = (2 * mx * my + c1) * (2 * sxy + c2) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return 1 - s.mean()


def torch_loss(P, T, opt, Hs, k, mask=None, ssim_weight=0.0):
    """P: dict of FP64 leaf tensors (pre-activation), T [L, C, H, W]."""
    H, W, C = opt.H, opt.W, opt.C
    mx = 0.5 * (torch.tanh(P["mean_pre"][:, 0]) + 1.0) * W
    my = 0.5 * (torch.tanh(P["mean_pre"][:, 1]) + 1.0) * H
    sx = torch.exp(P["log_scale"][:, 0]) + 0.1
    sy = torch.exp(P["log_scale"][:, 1]) + 0.1
    c, s = torch.cos(P["rotation"]), torch.sin(P["rotation"])
    s00 = sx * sx * c * c + sy * sy * s * s + 0.1
    s01 = (sx * sx - sy * sy) * c * s
    s11 = sx * sx * s * s + sy * sy * c * c + 0.1
    det = torch.clamp(s00 * s11 - s01 * s01, min=1e-10)
    i00, i01, i11 = s11 / det, -s01 / det, s00 / det
    alpha = torch.sigmoid(P["opacity_pre"])
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    dx = xs[None] - mx[:, None, None]
    dy = ys[None] - my[:, None, None]
    q = i00[:, None, None] * dx * dx + 2 * i01[:, None, None] * dx * dy + i11[:, None, None] * dy * dy
    G = torch.exp(torch.clamp(-0.5 * q, min=-50.0))
    if k > 0:
        G = torch.where(q <= k * k, G, torch.zeros_like(G))
    wgt = alpha[:, None, None] * G                                   # [N, H, W]
    amp, ph = P["amplitude"], P["phase"]                             # [N, C]
    re = torch.einsum("nc,nhw->chw", amp * torch.cos(ph), wgt)
    im = torch.einsum("nc,nhw->chw", amp * torch.sin(ph), wgt)
    field = torch.complex(re, im)
    spec = torch.fft.fft2(field, s=(opt.Hp, opt.Wp))                 # zero-extended at the end
    u = torch.fft.ifft2(spec[None] * Hs)[..., :H, :W]                # [L, C, H, W]
    I = u.real ** 2 + u.imag ** 2
    r = I - T
    n = I.numel()
    extra = ssim_weight * torch_ssim(I, T) if ssim_weight else 0.0
    if mask is None:
        return torch.sum(r * r) / n + extra
    Mk = mask[:, None]                                               # [L, 1, H, W]
    return (torch.sum(r * r) + torch.sum((I * Mk - T * Mk) ** 2)
            + torch.sum((I * T - T * T) ** 2)) / n + extra


@pytest.mark.parametrize("case", [
    dict(C=2, zs=[3e-3], k=3.0, mask=False),
    dict(C=1, zs=[2e-3, -4e-3], k=3.0, mask=True),
    dict(C=1, zs=[3e-3], k=0.0, mask=False),  # unbounded support: the exponent clamp binds
    # the paper's final loss: L_recon + 0.005 L_SSIM
    dict(C=2, zs=[2e-3, 5e-3], k=3.0, mask=True, ssim=0.005),
])
def test_adjoint_matches_autodiff(O, case):
    H, W, n = 20, 28, 30
    Hp, Wp = 40, 56
    C, zs, k = case["C"], case["zs"], case["k"]
    lambdas = [639e-9, 473e-9][:C]
    L = len(zs)
    p = synth.params(91, n, H, W, C)
    T = synth.target(92, C, H, W, L=L) * np.float32(0.5)
    mask = (np.random.default_rng(93).uniform(0, 1, (L, H, W)) > 0.5).astype(np.float32) \
        if case["mask"] else None
    opt = O.Optics(H, W, C, Hp, Wp, 8e-6, lambdas, zs, k=k)
    ssim = case.get("ssim", 0.0)
    ref = O.forward_backward(p, T, opt, mask=mask, ssim_weight=ssim)
    Hs = torch.from_numpy(np.stack([np.stack([O.transfer(Hp, Wp, 8e-6, lam, z) for lam in lambdas])
                                    for z in zs]))                   # [L, C, Hp, Wp]
    P = {key: torch.tensor(np.asarray(p[key], dtype=np.float64), requires_grad=True)
         for key in KEYS}
    loss = torch_loss(P, torch.from_numpy(T.astype(np.float64)), opt, Hs, k,
                      None if mask is None else torch.from_numpy(mask.astype(np.float64)),
                      ssim_weight=ssim)
    assert abs(loss.item() - ref["loss"]) <= 1e-12 * ref["loss"]
    loss.backward()
    for key in KEYS:
        g, r = P[key].grad.numpy(), ref["grads"][key]
        err = np.linalg.norm(g - r) / np.linalg.norm(r)
        assert err <= 1e-9, (key, err)
