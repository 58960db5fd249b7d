"""Pins for the oracle's Adan step (Xie et al., Algorithm 1, bias-corrected):
the first-step closed form, a hand-unrolled second step, and the reduction to
Adam (with the third decay rate) when the gradient does not change."""
import numpy as np


def test_first_step_closed_form(O):
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    p1, m, d, s, gp = O.adan(p0, g, z, z, z, z, 1, 1e-2)
    # m_hat = g, d = 0, s_hat = g^2: a signed step of lr
    assert np.allclose(p1, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.array_equal(gp, g) and np.array_equal(d, z)


def test_second_step_by_hand(O):
    # scalar, b = (0.5, 0.5, 0.5), lr 1, eps 0: g1 = 1, g2 = 3
    p, m, d, s, gp = O.adan(0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1, 1.0, 0.5, 0.5, 0.5, 0.0)
    # t=1: m = .5, d = 0, s = .5; m_hat = 1, s_hat = 1 -> p = -1
    assert (p, m, d, s) == (-1.0, 0.5, 0.0, 0.5)
    p, m, d, s, gp = O.adan(p, 3.0, m, d, s, gp, 2, 1.0, 0.5, 0.5, 0.5, 0.0)
    # t=2: diff = 2; m = .25 + 1.5 = 1.75; d = 0 + 1 = 1; u = 3 + 1 = 4; s = .25 + 8 = 8.25
    # m_hat = 1.75 / .75; d_hat = 1 / .75; s_hat = 8.25 / .75 = 11
    assert (m, d, s) == (1.75, 1.0, 8.25)
    expect = -1.0 - (1.75 / 0.75 + 0.5 * (1.0 / 0.75)) / np.sqrt(11.0)
    assert abs(p - expect) < 1e-15


def test_constant_gradient_is_adam(O):
    rng = np.random.default_rng(1)
    g = rng.standard_normal(40)
    pa = pb = rng.standard_normal(40)
    ma = va = np.zeros(40)
    mb = db = sb = gp = np.zeros(40)
    for t in range(1, 6):
        pa, ma, va = O.adam(pa, g, ma, va, t, 1e-3, beta1=0.98, beta2=0.99)
        pb, mb, db, sb, gp = O.adan(pb, g, mb, db, sb, gp, t, 1e-3)
        assert np.array_equal(db, np.zeros(40))
    assert np.allclose(pa, pb, rtol=0, atol=1e-14)
