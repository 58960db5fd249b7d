"""Pins for the oracle of the POH conversion (Sec. 3.3): the double-phase
identity, the reduction of L_extract when both holograms agree, and its
gradients against finite differences and torch.autograd of a separately
written loss."""
import numpy as np
import torch

from oracle import poh as P


def test_dpac_phasor_average_is_the_normalised_field():
    rng = np.random.default_rng(1)
    C, H, W = 2, 6, 8
    # a field constant over horizontal pairs (2k, 2k + 1): neighbours of opposite parity
    base = rng.standard_normal((C, H, W // 2)) + 1j * rng.standard_normal((C, H, W // 2))
    f = np.repeat(base, 2, axis=2)
    ph = P.dpac(f)
    avg = 0.5 * (np.exp(1j * ph[:, :, 0::2]) + np.exp(1j * ph[:, :, 1::2]))
    amax = np.abs(f).reshape(C, -1).max(axis=1)
    want = base / amax[:, None, None]
    assert np.max(np.abs(avg - want)) < 1e-12
    # the checkerboard: even cells take phi + arccos(A_n)
    A = np.abs(f) / amax[:, None, None]
    assert abs(ph[0, 0, 0] - (np.angle(f[0, 0, 0]) + np.arccos(A[0, 0, 0]))) < 1e-12
    assert abs(ph[0, 0, 1] - (np.angle(f[0, 0, 1]) - np.arccos(A[0, 0, 1]))) < 1e-12
    assert abs(ph[0, 1, 0] - (np.angle(f[0, 1, 0]) - np.arccos(A[0, 1, 0]))) < 1e-12


def test_dpac_unit_amplitude_and_zero_field():
    phi = np.random.default_rng(2).uniform(-3, 3, (1, 4, 5))
    # |exp(j phi)| is 1 to rounding, and arccos(1 - e) ~ sqrt(2 e): 1e-8 here
    assert np.max(np.abs(P.dpac(np.exp(1j * phi)) - phi)) < 1e-7
    z = P.dpac(np.zeros((1, 3, 3), np.complex128))
    # A_n = 0: the two phasors are +-j, their mean is 0
    assert np.allclose(np.abs(z), np.pi / 2)


def test_extract_loss_when_both_holograms_agree():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((2, 1, 5, 6)) + 1j * rng.standard_normal((2, 1, 5, 6))
    T = rng.uniform(0, 1, (2, 1, 5, 6))
    M = (rng.uniform(0, 1, (2, 5, 6)) > 0.5).astype(float)
    from oracle import oracle as O
    l, gu, gur = P.extract_loss(u, u, T, M)
    lr, _, g = O.recon(u, T, M)
    assert abs(l - 2 * lr) < 1e-12
    # the comparison and field terms have zero (sub)gradient at u = u_rand
    assert np.max(np.abs(gu - g)) < 1e-12 and np.max(np.abs(gur - g)) < 1e-12


def torch_extract(u, ur, T, M, lc=0.1, lf=0.01):
    I, Ir = u.abs() ** 2, ur.abs() ** 2
    w = 1 + M ** 2 + T ** 2
    rec = lambda X: ((X - T) ** 2 * w).mean()
    d = u - ur
    return rec(I) + rec(Ir) + lc * ((I - Ir) ** 2).mean() + lf * (d.real.abs() + d.imag.abs()).mean()


def test_extract_gradients_against_autodiff_and_fd():
    rng = np.random.default_rng(4)
    shape = (2, 2, 4, 5)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ur = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    T = rng.uniform(0, 1, shape)
    M = (rng.uniform(0, 1, (2, 4, 5)) > 0.5).astype(float)
    l, gu, gur = P.extract_loss(u, ur, T, M)
    tu = torch.tensor(u, requires_grad=True)
    tr = torch.tensor(ur, requires_grad=True)
    tl = torch_extract(tu, tr, torch.tensor(T), torch.tensor(M)[:, None])
    tl.backward()
    assert abs(tl.item() - l) < 1e-12 * max(1.0, abs(l))
    # torch's gradient of a real loss in a complex tensor is dL/dRe + j dL/dIm
    assert np.max(np.abs(tu.grad.numpy() - gu)) < 1e-12
    assert np.max(np.abs(tr.grad.numpy() - gur)) < 1e-12
    h = 1e-7
    for idx in [(0, 0, 1, 2), (1, 1, 3, 4)]:
        for part in (1.0, 1j):
            up, um = u.copy(), u.copy()
            up[idx] += part * h
            um[idx] -= part * h
            fd = (P.extract_loss(up, ur, T, M)[0] - P.extract_loss(um, ur, T, M)[0]) / (2 * h)
            an = gu[idx].real if part == 1.0 else gu[idx].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def test_phase_gradient_against_fd():
    rng = np.random.default_rng(5)
    phi = rng.uniform(-3, 3, (1, 3, 4))
    g = rng.standard_normal((1, 3, 4)) + 1j * rng.standard_normal((1, 3, 4))
    # L = Re <g, exp(j phi)> has dL/dH = g
    f = lambda p: np.sum((np.conj(g) * np.exp(1j * p)).real)
    an = P.phase_grad(phi, g)
    for idx in [(0, 0, 0), (0, 2, 3)]:
        pp, pm = phi.copy(), phi.copy()
        pp[idx] += 1e-6
        pm[idx] -= 1e-6
        assert abs((f(pp) - f(pm)) / 2e-6 - an[idx]) < 1e-8
