"""GPU parity of the POH conversion (include/cgh_poh.h,
cgh_propagate_field_adjoint) against the FP64 oracle (oracle/poh.py), through
the C ABI."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import poh as OP
from paper_2511_15022_amd import binding, poh, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_smooth_poh_matches_oracle():
    rng = np.random.default_rng(1)
    C, H, W = 3, 37, 53
    f = (rng.standard_normal((C, H, W)) + 1j * rng.standard_normal((C, H, W))).astype(np.complex64)
    phase, hs = poh.smooth(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    ref = OP.dpac(f.astype(np.complex128))
    # compare phasors (phases wrap); FP32 arccos near A_n = 1 is the weakest step
    e = rel(np.exp(1j * phase.cpu().numpy()), np.exp(1j * ref))
    say("dpac phasor rel", e)
    assert e <= 1e-5
    assert rel(hs.cpu().numpy(), np.exp(1j * phase.cpu().numpy().astype(np.float64))) <= 1e-6


def test_phase_field_and_gradient():
    rng = np.random.default_rng(2)
    n = 1000
    ph = rng.uniform(-7, 7, n).astype(np.float32)
    g = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    L = binding.lib()
    s = torch.cuda.current_stream().cuda_stream
    tp, tg = torch.from_numpy(ph).cuda(), torch.from_numpy(g).cuda()
    out = torch.empty(n, dtype=torch.complex64, device="cuda")
    gp = torch.empty(n, dtype=torch.float32, device="cuda")
    assert L.cgh_poh_field(tp.data_ptr(), n, out.data_ptr(), s) == 0
    assert L.cgh_poh_phase_grad(tp.data_ptr(), tg.data_ptr(), n, gp.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), np.exp(1j * ph.astype(np.float64))) <= 1e-6
    assert rel(gp.cpu().numpy(), OP.phase_grad(ph, g)) <= 1e-6


@pytest.mark.parametrize("masked", [False, True])
def test_extract_seed_matches_oracle(masked):
    rng = np.random.default_rng(3)
    L, C, H, W = 2, 3, 13, 17
    shape = (L, C, H, W)
    u = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    ur = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    T = rng.uniform(0, 1, shape).astype(np.float32)
    M = (rng.uniform(0, 1, (L, H, W)) > 0.5).astype(np.float32) if masked else None
    n = L * C * H * W
    Lb = binding.lib()
    gu = torch.empty(shape, dtype=torch.complex64, device="cuda")
    gur = torch.empty_like(gu)
    part = torch.empty(Lb.cgh_poh_extract_partials(n), dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    tu, tur, tT = (torch.from_numpy(a).cuda() for a in (u, ur, T))
    tM = torch.from_numpy(M).cuda() if masked else None
    assert Lb.cgh_poh_extract_seed(tu.data_ptr(), tur.data_ptr(), tT.data_ptr(),
                                   tM.data_ptr() if masked else None, L, C, H, W, 0.1, 0.01,
                                   gu.data_ptr(), gur.data_ptr(), part.data_ptr(),
                                   loss.data_ptr(), torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    l, g1, g2 = OP.extract_loss(u.astype(np.complex128), ur.astype(np.complex128), T, M)
    say("extract loss", loss.item(), l)
    assert abs(loss.item() - l) <= 1e-6 * l
    assert rel(gu.cpu().numpy(), g1) <= 1e-5
    assert rel(gur.cpu().numpy(), g2) <= 1e-5


def test_field_adjoint_matches_oracle():
    rng = np.random.default_rng(4)
    H, W, C, lams, zs = 40, 56, 2, [639e-9, 473e-9], [2e-3, -3e-3]
    ctx = binding.Context(H, W, C, 8e-6, lams, zs, pad=(80, 120), max_gaussians=1)
    g = (rng.standard_normal((2, C, H, W)) + 1j * rng.standard_normal((2, C, H, W))).astype(np.complex64)
    out = ctx.propagate_field_adjoint(torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    opt = O.Optics(H, W, C, 80, 120, 8e-6, lams, zs)
    ref = O.propagate_adjoint(g.astype(np.complex128), opt)
    e = rel(out.cpu().numpy(), ref)
    say("field adjoint rel", e)
    assert e <= 1e-4


def test_random_poh_step_gradients_match_oracle():
    """One joint step of the Random POH (two planes, focal masks): the
    gradients of the Gaussians' parameters and of the phase against the
    oracle's composition (propagation, L_extract, adjoint propagation,
    rasterizer adjoint, phase gradient)."""
    H, W, C, n = 40, 56, 2, 300
    lams, zs = [639e-9, 473e-9], [3e-3, 5e-3]
    p = synth.params(41, n, H, W, C)
    T = synth.target(42, C, H, W, L=2) * np.float32(0.5)
    M = (np.random.default_rng(43).uniform(0, 1, (2, H, W)) > 0.5).astype(np.float32)
    ctx = binding.Context(H, W, C, 8e-6, lams, zs, pad=(80, 120), max_gaussians=n)
    rp = poh.RandomPOH(ctx, binding.pack(p, device="cuda"), n, torch.from_numpy(T).cuda(),
                       torch.from_numpy(M).cuda(), seed=44)
    phase = rp.phase.cpu().numpy().astype(np.float64)
    rp.gradients()
    torch.cuda.synchronize()
    opt = O.Optics(H, W, C, 80, 120, 8e-6, lams, zs)
    field = O.raster(p, opt)
    u = O.propagate(field, opt)
    ur = O.propagate(np.exp(1j * phase), opt)
    l, gu, gur = OP.extract_loss(u, ur, T, M)
    gfield = O.propagate_adjoint(gu, opt)
    grads = O.raster_adjoint(p, gfield, opt)
    gphase = OP.phase_grad(phase, O.propagate_adjoint(gur, opt))
    say("loss", rp.loss.item(), l)
    assert abs(rp.loss.item() - l) <= 1e-4 * l
    views = binding.unpack(rp.G.cpu(), n, C)
    for k in binding.PARAM_KEYS:
        e = rel(views[k].numpy(), grads[k])
        assert e <= 1e-3, (k, e)
    e = rel(rp.gphase.cpu().numpy(), gphase)
    say("phase gradient rel", e)
    assert e <= 1e-3
