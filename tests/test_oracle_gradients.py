"""Pins for the oracle's analytic adjoint (supplementary Backward Pass, items
1-7, and the BLASM backward pass): FP64 central finite differences of the
whole forward (raster -> pad -> propagate -> |u|^2 -> L_MSE) with the k-sigma
support held at the base point, and the textbook Adam update."""
import numpy as np
import pytest

from paper_2511_15022_amd import synth

GROUPS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")


def problem(O, H=24, W=32, C=2, n=24, L=2, k=3.0, flags=0, seed=7):
    p = synth.params(seed, n, H, W, C)
    opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, [639e-9, 473e-9][:C], [2e-3, 6e-3][:L], k=k,
                   flags=flags)
    # target scaled to the field's intensity range so the loss is not trivial
    T = synth.target(seed + 1, C, H, W, L=L) * 0.3
    return p, opt, T


@pytest.mark.parametrize("k, flags", [(3.0, 0), (0.0, 0), (3.0, 2)])
def test_analytic_gradient_matches_finite_differences(O, k, flags):
    p, opt, T = problem(O, k=k, flags=flags)
    fb = O.forward_backward(p, T, opt)
    rng = np.random.default_rng(int(k * 10) + flags)
    for key in GROUPS:
        g = fb["grads"][key].reshape(-1)
        scale = np.max(np.abs(g))
        assert scale > 0
        for idx in rng.choice(g.size, size=4, replace=False):
            fd = O.fd_gradient(p, T, opt, key, int(idx))
            assert abs(fd - g[idx]) <= 1e-6 * scale, (key, idx, fd, g[idx])


def test_loss_gradient_wrt_field_by_finite_differences(O):
    """dL/dU0 (propagation adjoint + intensity/MSE derivative) against central
    differences in the real and imaginary part of single field entries."""
    p, opt, T = problem(O, n=10)
    field = O.raster(p, opt)

    def loss(f):
        return O.mse(O.propagate(f, opt), T)[0]

    u = O.propagate(field, opt)
    _, _, gu = O.mse(u, T)
    gf = O.propagate_adjoint(gu, opt)
    h = 1e-6
    for (c, j, i) in [(0, 3, 4), (1, 12, 20), (0, 23, 31)]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            fp = field.copy()
            fm = field.copy()
            fp[c, j, i] += h * unit
            fm[c, j, i] -= h * unit
            fd = (loss(fp) - loss(fm)) / (2 * h)
            an = gf[c, j, i].real if part == "re" else gf[c, j, i].imag
            assert abs(fd - an) <= 1e-7 * np.max(np.abs(gf)), (c, j, i, part, fd, an)


def test_frozen_support_reproduces_plain_forward(O):
    p, opt, T = problem(O, n=30)
    a = O.raster(p, opt)
    b = O.raster(p, opt, support=p)
    assert np.array_equal(a, b)


def test_adam_first_step_and_library(O):
    """Kingma & Ba: at t = 1 the bias-corrected update is -lr g / (|g| + eps);
    later steps agree with torch.optim.Adam run in float64 on the CPU."""
    import torch
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    g = rng.standard_normal(50)
    p1, m, v = O.adam(p0, g, m, v, 1, lr)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    optim = torch.optim.Adam([tp], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    pp, mm, vv = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        gt = rng.standard_normal(50)
        tp.grad = torch.tensor(gt)
        optim.step()
        pp, mm, vv = O.adam(pp, gt, mm, vv, t, lr)
    assert np.allclose(tp.detach().numpy(), pp, rtol=0, atol=1e-14)
