"""Pins the oracle's hand-derived adjoint (supplementary Backward Pass, chained
through the activations of Sec. 3.1) to automatic differentiation: the forward
is restated here from the paper's formulas with torch operations in FP64
(brute force over every pixel and Gaussian, FFT-based propagation with the
band-limited transfer function, L_MSE or L_recon), and torch.autograd
differentiates it.  The support indicator q <= k^2 is piecewise constant, so
both sides differentiate the same function; agreement is to rounding."""
import numpy as np
import pytest
import torch

from paper_2511_15022_amd import synth

KEYS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")


def torch_loss(P, T, opt, Hs, k, mask=None):
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
    if mask is None:
        return torch.sum(r * r) / n
    Mk = mask[:, None]                                               # [L, 1, H, W]
    return (torch.sum(r * r) + torch.sum((I * Mk - T * Mk) ** 2) + torch.sum((I * T - T * T) ** 2)) / n


@pytest.mark.parametrize("case", [
    dict(C=2, zs=[3e-3], k=3.0, mask=False),
    dict(C=1, zs=[2e-3, -4e-3], k=3.0, mask=True),
    dict(C=1, zs=[3e-3], k=0.0, mask=False),  # unbounded support: the exponent clamp binds
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
    ref = O.forward_backward(p, T, opt, mask=mask)
    Hs = torch.from_numpy(np.stack([np.stack([O.transfer(Hp, Wp, 8e-6, lam, z) for lam in lambdas])
                                    for z in zs]))                   # [L, C, Hp, Wp]
    P = {key: torch.tensor(np.asarray(p[key], dtype=np.float64), requires_grad=True)
         for key in KEYS}
    loss = torch_loss(P, torch.from_numpy(T.astype(np.float64)), opt, Hs, k,
                      None if mask is None else torch.from_numpy(mask.astype(np.float64)))
    assert abs(loss.item() - ref["loss"]) <= 1e-12 * ref["loss"]
    loss.backward()
    for key in KEYS:
        g, r = P[key].grad.numpy(), ref["grads"][key]
        err = np.linalg.norm(g - r) / np.linalg.norm(r)
        assert err <= 1e-9, (key, err)
