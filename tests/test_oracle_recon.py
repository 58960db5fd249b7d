"""Pins for the oracle's reconstruction loss (Sec. 3.2, L_recon): a hand sum,
the reduction to L_MSE when the mask and target vanish, central differences
of the loss in the real and imaginary parts of u, and FP64 finite
differences of the whole chain (raster -> propagate -> L_recon) in the
pre-activation parameters."""
import numpy as np

from paper_2511_15022_amd import synth


def test_hand_sum(O):
    # one plane, one channel, two pixels: u = (1 + j, 2), T = (1, 3), M = (1, 0)
    # I = (2, 4); I - T = (1, 1); I M - T M = (1, 0); I T - T T = (1, 3)
    # sum of squares 2 + 1 + 10 = 13 over 2 elements
    u = np.array([1 + 1j, 2 + 0j]).reshape(1, 1, 1, 2)
    T = np.array([1.0, 3.0]).reshape(1, 1, 1, 2)
    M = np.array([1.0, 0.0]).reshape(1, 1, 2)
    loss, I, g = O.recon(u, T, M)
    assert loss == 6.5
    assert np.array_equal(I.ravel(), [2.0, 4.0])
    # dL/dI = 2 (I - T)(1 + M^2 + T^2) / 2 = (3, 10); grad_u = 2 dL/dI u
    assert np.allclose(g.ravel(), [6 * (1 + 1j), 40.0])


def test_reduces_to_mse_without_mask_and_target(O):
    rng = np.random.default_rng(0)
    u = rng.standard_normal((2, 3, 5, 7)) + 1j * rng.standard_normal((2, 3, 5, 7))
    T = np.zeros((2, 3, 5, 7))
    M = np.zeros((2, 5, 7))
    a = O.recon(u, T, M)
    b = O.mse(u, T)
    assert a[0] == b[0]
    assert np.array_equal(a[2], b[2])


def test_grad_u_by_central_differences(O):
    rng = np.random.default_rng(1)
    u = rng.standard_normal((2, 2, 4, 5)) + 1j * rng.standard_normal((2, 2, 4, 5))
    T = rng.uniform(0, 1, (2, 2, 4, 5))
    M = (rng.uniform(0, 1, (2, 4, 5)) > 0.5).astype(float)
    _, _, g = O.recon(u, T, M)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 3, 4), (0, 1, 2, 3), (1, 0, 1, 1)]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            up = u.copy(); um = u.copy()
            up[idx] += h * unit; um[idx] -= h * unit
            fd = (O.recon(up, T, M)[0] - O.recon(um, T, M)[0]) / (2 * h)
            an = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (idx, part, fd, an)


def test_parameter_gradients_by_finite_differences(O):
    H, W, C, n = 24, 32, 2, 20
    p = synth.params(17, n, H, W, C)
    opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, [639e-9, 473e-9], [2e-3, 5e-3])
    T = synth.target(18, C, H, W, L=2) * 0.3
    M = (np.random.default_rng(19).uniform(0, 1, (2, H, W)) > 0.6).astype(np.float64)
    fb = O.forward_backward(p, T, opt, mask=M)
    rng = np.random.default_rng(20)
    for key in ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre"):
        g = fb["grads"][key].reshape(-1)
        scale = np.max(np.abs(g))
        for idx in rng.choice(g.size, size=3, replace=False):
            fd = O.fd_gradient(p, T, opt, key, int(idx), mask=M)
            assert abs(fd - g[idx]) <= 1e-6 * scale, (key, idx, fd, g[idx])
