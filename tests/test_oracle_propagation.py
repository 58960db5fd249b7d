"""Pins for the oracle's propagation (Alg. 1 ZeroPad + MultiPlanePropagate;
supplementary BLASM forward and backward): identities of free-space
propagation that hold exactly on the discrete grid."""
import numpy as np
import pytest


def optics(O, H, W, Hp, Wp, zs, lambdas=(515e-9,), pitch=8e-6):
    return O.Optics(H, W, len(lambdas), Hp, Wp, pitch, list(lambdas), list(zs))


def rand_field(rng, C, H, W):
    return rng.standard_normal((C, H, W)) + 1j * rng.standard_normal((C, H, W))


def test_zero_distance_is_identity(O):
    rng = np.random.default_rng(0)
    opt = optics(O, 20, 30, 40, 60, [0.0])
    x = rand_field(rng, 1, 20, 30)
    u = O.propagate(x, opt)[0]
    assert np.max(np.abs(u - x)) < 1e-13


def test_forward_then_backward_distance_returns_input_on_full_grid(O):
    """Without padding the transfer function acts on the whole periodic grid;
    inside the band |H| = 1 and H(-z) = H(z)*, so P_{-z} P_z = identity."""
    rng = np.random.default_rng(1)
    x = rand_field(rng, 1, 48, 64)
    fwd = optics(O, 48, 64, 48, 64, [5e-3])
    bwd = optics(O, 48, 64, 48, 64, [-5e-3])
    u = O.propagate(x, fwd)[0]
    back = O.propagate(u, bwd)[0]
    assert np.max(np.abs(back - x)) < 1e-12
    # Parseval: the unpadded propagation is unitary when no bin is cut
    assert abs(np.linalg.norm(u) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def test_band_limit_projects_on_round_trip(O):
    """With the stress geometry the band limit removes bins: the round trip is
    the orthogonal projector onto the kept band (idempotent, norm-reducing)."""
    rng = np.random.default_rng(2)
    x = rand_field(rng, 1, 64, 64)
    fwd = optics(O, 64, 64, 64, 64, [300e-3])
    bwd = optics(O, 64, 64, 64, 64, [-300e-3])
    once = O.propagate(O.propagate(x, fwd)[0], bwd)[0]
    twice = O.propagate(O.propagate(once, fwd)[0], bwd)[0]
    assert np.max(np.abs(twice - once)) < 1e-12
    assert np.linalg.norm(once) < np.linalg.norm(x)
    # orthogonality: (x - Px) is orthogonal to Px
    assert abs(np.vdot(x - once, once)) < 1e-10 * np.linalg.norm(x) ** 2


def test_plane_wave_is_eigenfunction(O):
    """A grid-periodic plane wave at bin (ky, kx) leaves the unpadded propagator
    multiplied by H[ky, kx]."""
    H, W = 32, 40
    ky, kx = 3, 37
    jj, ii = np.mgrid[0:H, 0:W]
    x = np.exp(2j * np.pi * (kx * ii / W + ky * jj / H))[None]
    opt = optics(O, H, W, H, W, [4e-3], lambdas=(639e-9,))
    u = O.propagate(x, opt)[0]
    h = O.transfer(H, W, 8e-6, 639e-9, 4e-3)[ky, kx]
    assert np.max(np.abs(u - h * x)) < 1e-12


def test_interior_translation_commutes(O):
    """Propagation is a convolution: translating a compactly supported input
    (that stays clear of the padding edges) translates the output."""
    rng = np.random.default_rng(3)
    x = np.zeros((1, 40, 40), complex)
    x[0, 15:22, 12:20] = rng.standard_normal((7, 8)) + 1j * rng.standard_normal((7, 8))
    xs = np.roll(x, (3, -2), axis=(1, 2))
    opt = optics(O, 40, 40, 80, 80, [1e-3])
    u = O.propagate(x, opt)[0, 0]
    us = O.propagate(xs, opt)[0, 0]
    # compare on the region where neither shifted copy touches the crop edge
    ref = np.roll(u, (3, -2), axis=(0, 1))
    assert np.max(np.abs(us[5:35, 5:35] - ref[5:35, 5:35])) < 1e-12


@pytest.mark.parametrize("shape", [(24, 40, 48, 80), (30, 20, 45, 40), (16, 16, 32, 32)])
def test_adjoint_dot_product(O, shape):
    """Re<P x, y> = Re<x, P^H y> with P = crop o IFFT o H o FFT o pad, summed
    over planes and channels (supplementary BLASM backward: conjugate H, same
    band limit)."""
    H, W, Hp, Wp = shape
    rng = np.random.default_rng(H + W)
    opt = O.Optics(H, W, 2, Hp, Wp, 8e-6, [639e-9, 473e-9], [3e-3, 200e-3])
    x = rand_field(rng, 2, H, W)
    y = rng.standard_normal((2, 2, H, W)) + 1j * rng.standard_normal((2, 2, H, W))
    Px = O.propagate(x, opt)
    PHy = O.propagate_adjoint(y, opt)
    lhs = np.real(np.vdot(y, Px))
    rhs = np.real(np.vdot(PHy, x))
    assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(y) * np.linalg.norm(x))


def test_padding_is_centred(O):
    """A delta at the canvas centre stays centred: its intensity pattern is
    point-symmetric about the centre (centred zero-padding and crop)."""
    H = W = 33
    x = np.zeros((1, H, W), complex)
    x[0, 16, 16] = 1.0
    opt = optics(O, H, W, 66, 66, [2e-3])
    I = np.abs(O.propagate(x, opt)[0, 0]) ** 2
    assert np.max(np.abs(I - I[::-1, ::-1])) < 1e-14
