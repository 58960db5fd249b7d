"""Pins for the oracle's SSIM term (Wang et al. 2004; the L_SSIM of the
paper's final loss, Sec. 3.2): identities and closed forms of the definition,
its gradient against torch.autograd of a separately written SSIM (separable
conv2d filtering, not sliding windows), and finite differences."""
import numpy as np
import torch

C1, C2 = 0.01 ** 2, 0.03 ** 2


def test_window(O):
    w = O.ssim_window()
    assert w.shape == (11,) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-18) and w.argmax() == 5
    # ratio of neighbouring weights of a Gaussian of standard deviation 1.5
    assert abs(w[5] / w[6] - np.exp(1.0 / (2 * 1.5 ** 2))) < 1e-14


def test_identity_and_constants(O):
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (20, 23))
    assert np.abs(O.ssim_parts(x, x)["ssim"] - 1.0).max() < 1e-12
    I = rng.uniform(0, 1, (2, 1, 16, 17))
    loss, g = O.ssim_loss(I, I)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-9
    # constant images: sigmas vanish, SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    s = O.ssim_parts(np.full((12, 12), a), np.full((12, 12), b))["ssim"]
    assert s.shape == (2, 2)
    assert np.abs(s - (2 * a * b + C1) / (a * a + b * b + C1)).max() < 1e-12


def test_offset_reduces_to_luminance(O):
    """y = x + c: equal contrast and structure, so SSIM is the luminance term of
    the window means; the means here come from separable 1-D filtering."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 0.5, (19, 25))
    c = 0.2
    w = O.ssim_window()
    rows = np.stack([np.convolve(r, w[::-1], mode="valid") for r in x])
    mu = np.stack([np.convolve(col, w[::-1], mode="valid") for col in rows.T]).T
    expect = (2 * mu * (mu + c) + C1) / (mu * mu + (mu + c) ** 2 + C1)
    assert np.abs(O.ssim_parts(x, x + c)["ssim"] - expect).max() < 1e-12


def torch_ssim_loss(I, T):
    """1 - mean SSIM with separable conv2d filtering (written independently)."""
    i = torch.arange(11, dtype=torch.float64) - 5
    w = torch.exp(-(i * i) / (2 * 1.5 ** 2))
    w = w / w.sum()
    L, C, H, W = I.shape
    x = I.reshape(L * C, 1, H, W)
    y = T.reshape(L * C, 1, H, W)

    def f(a):
        a = torch.nn.functional.conv2d(a, w.view(1, 1, 1, 11))
        return torch.nn.functional.conv2d(a, w.view(1, 1, 11, 1))

    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    s = (2 * mx * my + C1) * (2 * sxy + C2) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return 1 - s.mean()


def test_gradient_against_autodiff_and_fd(O):
    rng = np.random.default_rng(3)
    I = rng.uniform(0, 1, (2, 2, 15, 18))
    T = np.clip(I + 0.2 * rng.standard_normal(I.shape), 0, 1)
    loss, g = O.ssim_loss(I, T)
    It = torch.tensor(I, requires_grad=True)
    lt = torch_ssim_loss(It, torch.tensor(T))
    lt.backward()
    assert abs(lt.item() - loss) < 1e-13
    assert np.linalg.norm(It.grad.numpy() - g) / np.linalg.norm(g) < 1e-11
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 7, 9), (0, 1, 14, 17), (1, 0, 5, 0)]:
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (O.ssim_loss(Ip, T)[0] - O.ssim_loss(Im, T)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx])) + 1e-9, (idx, fd, g[idx])
