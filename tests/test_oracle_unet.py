"""Pins for the oracle of the learned initialiser's network: the convolution
against explicit sums, its adjoints by the dot-product identity, pooling and
upsampling adjoints, BF16 rounding on hand-picked values, the network's
backward and the lattice gather against FP64 finite differences."""
import numpy as np
import pytest

from oracle import unet as U


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, 1 + 3 * 2.0 ** -8,
                  -2.5, 3.0e38, 1e-40], np.float64)
    r = U.bf16(v)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2.0 ** -7
    # 1 + 3 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: the even one is 1 + 2^-6
    assert r[3] == 1 + 2.0 ** -6
    assert r[4] == -2.5
    # 8 significant bits everywhere
    x = np.random.default_rng(0).standard_normal(1000) * 100
    rx = U.bf16(x)
    assert np.all(np.abs(rx - x) <= np.abs(x) * 2.0 ** -8 + 1e-300)
    assert np.array_equal(U.bf16(rx), rx)


def test_conv_matches_explicit_sums():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = U.conv3x3(x, w, b)
    ref = np.zeros((5, 6, 4))
    for y in range(5):
        for xx in range(6):
            for co in range(4):
                s = b[co]
                for ky in range(3):
                    for kx in range(3):
                        yy, xq = y + ky - 1, xx + kx - 1
                        if 0 <= yy < 5 and 0 <= xq < 6:
                            for ci in range(3):
                                s += x[yy, xq, ci] * w[co, ky, kx, ci]
                ref[y, xx, co] = s
    assert np.max(np.abs(out - ref)) < 1e-12


def test_conv_adjoints_dot_product():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((7, 9, 5))
    w = rng.standard_normal((6, 3, 3, 5))
    gy = rng.standard_normal((7, 9, 6))
    gx, gw, gb = U.conv3x3_backward(x, w, gy)
    lhs = np.sum(U.conv3x3(x, w) * gy)
    assert abs(lhs - np.sum(x * gx)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(w * gw)) < 1e-10 * abs(lhs)
    assert np.allclose(gb, gy.sum(axis=(0, 1)), rtol=0, atol=1e-12)
    # bias: d/db of <conv(x, w, b), gy> is the sum of gy
    b = rng.standard_normal(6)
    d = np.sum(U.conv3x3(x, w, b) * gy) - lhs
    assert abs(d - np.dot(b, gb)) < 1e-10 * max(1.0, abs(d))


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 6, 3))
    g = rng.standard_normal((4, 3, 3))
    assert abs(np.sum(U.pool2(x) * g) - np.sum(x * U.pool2_adjoint(g))) < 1e-12
    y = rng.standard_normal((8, 6, 3))
    assert abs(np.sum(U.up2(g) * y) - np.sum(g * U.up2_adjoint(y))) < 1e-12
    assert np.allclose(U.pool2(np.full((4, 4, 2), 3.0)), 3.0)
    assert np.array_equal(U.pool2(U.up2(g)), g)


def small_net():
    arch = U.architecture(c_in=8, widths=(8, 16, 24), c_out=8)
    W = U.init_weights(arch, 5)
    rng = np.random.default_rng(6)
    for k in W:
        if k.endswith(".b"):
            W[k] = (0.1 * rng.standard_normal(W[k].shape)).astype(np.float32)
    return arch, W


def test_network_backward_matches_finite_differences():
    arch, W = small_net()
    rng = np.random.default_rng(7)
    x = rng.standard_normal((8, 12, 8))
    gout = rng.standard_normal((8, 12, 8))
    ident = lambda a: np.asarray(a, np.float64)
    Wd = {k: v.astype(np.float64) for k, v in W.items()}
    out, cache = U.forward(arch, Wd, x, q=ident)
    grads = U.backward(arch, Wd, cache, gout, q=ident)
    f = lambda Wp: np.sum(U.forward(arch, Wp, x, q=ident)[0] * gout)
    checked = 0
    for name in ("enc0a", "enc1b", "enc2a", "dec1a", "dec0a", "dec0b", "head", "enc2b.b",
                 "dec1a.b"):
        flat = Wd[name].reshape(-1)
        for idx in rng.choice(flat.size, 3, replace=False):
            h = 1e-6
            Wp = {k: v.copy() for k, v in Wd.items()}
            Wm = {k: v.copy() for k, v in Wd.items()}
            Wp[name].reshape(-1)[idx] += h
            Wm[name].reshape(-1)[idx] -= h
            fd = (f(Wp) - f(Wm)) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            scale = np.abs(grads[name]).max()
            assert abs(fd - an) <= 1e-6 * scale + 1e-9, (name, idx, fd, an)
            checked += 1
    assert checked == 27


@pytest.mark.parametrize("C", [1, 3])
def test_gather_adjoint_matches_finite_differences(C):
    H, W, gy, gx = 20, 30, 9, 13
    rng = np.random.default_rng(8)
    out = 0.3 * rng.standard_normal((H, W, 8 * C))
    gp = {"mean_pre": rng.standard_normal((gy * gx, 2)), "log_scale": rng.standard_normal((gy * gx, 2)),
          "rotation": rng.standard_normal(gy * gx), "amplitude": rng.standard_normal((gy * gx, C)),
          "phase": rng.standard_normal((gy * gx, C)), "opacity_pre": rng.standard_normal(gy * gx)}
    g = U.gather_adjoint(gp, out, H, W, gy, gx, C)

    def f(o):
        p = U.gather(o, H, W, gy, gx, C)
        return sum(np.sum(np.asarray(p[k]) * gp[k]) for k in gp)

    cy, cx = U.lattice(H, W, gy, gx)
    iy, ix = np.floor(cy).astype(int).reshape(-1), np.floor(cx).astype(int).reshape(-1)
    # every lattice point reads its own pixel, and no two share one
    assert len(set(zip(iy, ix))) == gy * gx
    for t in rng.choice(gy * gx, 6, replace=False):
        for ch in range(8 * C):
            o1, o2 = out.copy(), out.copy()
            o1[iy[t], ix[t], ch] += 1e-6
            o2[iy[t], ix[t], ch] -= 1e-6
            fd = (f(o1) - f(o2)) / 2e-6
            assert abs(fd - g[iy[t], ix[t], ch]) < 1e-5 * max(1.0, abs(fd))
    # pixels no lattice point reads get no gradient, nor do the unused
    # channels of the colour blocks after the first
    mask = np.ones((H, W), bool)
    mask[iy, ix] = False
    assert np.all(g[mask] == 0)
    for c in range(1, C):
        for k in (0, 1, 2, 3, 4, 7):
            assert np.all(g[:, :, 8 * c + k] == 0)
    # C = 1 reads channels 5 and 6 as the amplitude and phase
    p1 = U.gather(out, H, W, gy, gx, C)
    assert np.allclose(np.asarray(p1["amplitude"])[:, C - 1],
                       out[np.floor(cy).astype(int), np.floor(cx).astype(int)][..., 8 * (C - 1) + 5]
                       .reshape(-1) + 0.5)
