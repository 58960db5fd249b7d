"""GPU parity of the learned initialiser's network kernels (include/cgh_net.h)
against the FP64 oracle (oracle/unet.py), through the C ABI.  Inputs are BF16
on both sides, so the two differ only by FP32 against FP64 sums: the bar is
a relative L2 error of 1e-5 per output (FP32 accumulation over up to
9 x 384 terms), except where a sum is itself rounded to BF16 (one BF16 ulp,
2^-8 relative, at the elements where the two roundings differ)."""
import sys
import zlib

import numpy as np
import pytest
import torch

from oracle import unet as U
from paper_2511_15022_amd import binding

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def bf(shape, rng, scale=1.0):
    """A BF16 device tensor and its exact FP64 copy."""
    t = torch.from_numpy((rng.standard_normal(shape) * scale).astype(np.float32))
    t = t.to(torch.bfloat16)
    return t.cuda(), t.to(torch.float64).numpy()


def P(t):
    return None if t is None else t.data_ptr()


def stream():
    return torch.cuda.current_stream().cuda_stream


def check(st):
    assert st == 0, binding.lib().cgh_last_error().decode()


@pytest.mark.parametrize("case", [
    dict(H=19, W=23, c1=8, c2=0, up=False, cout=32, relu=True),     # ragged tiles
    dict(H=16, W=20, c1=32, c2=16, up=True, cout=64, relu=False),   # [up(x1), x2]
    dict(H=7, W=9, c1=64, c2=0, up=False, cout=128, relu=True),     # 4 blocks of 32
    dict(H=12, W=8, c1=256, c2=128, up=True, cout=128, relu=True),  # widest decoder input
    dict(H=9, W=13, c1=32, c2=0, up=False, cout=8, relu=False),     # the head: 8 of 32 channels
    # many workgroups of 256 pixels, the last one ragged; 24 input channels
    # (a half-filled last block of 16); [up(x1), x2] with 24 outputs
    dict(H=70, W=520, c1=24, c2=0, up=False, cout=32, relu=True),
    dict(H=38, W=300, c1=16, c2=16, up=True, cout=24, relu=False),
])
def test_conv_forward_and_adjoints(case):
    say("conv", case)
    rng = np.random.default_rng(zlib.crc32(str(sorted(case.items())).encode()))
    H, W, c1, c2, up, cout = case["H"], case["W"], case["c1"], case["c2"], case["up"], case["cout"]
    h1, w1 = (H // 2, W // 2) if up else (H, W)
    x1, x1n = bf((h1, w1, c1), rng)
    x2, x2n = bf((H, W, c2), rng) if c2 else (None, None)
    cin = c1 + c2
    w, wn = bf((cout, 3, 3, cin), rng, 1.0 / np.sqrt(9 * cin))
    b = torch.from_numpy(rng.standard_normal(cout).astype(np.float32)).cuda()
    out32 = torch.empty((H, W, cout), dtype=torch.float32, device="cuda")
    out16 = torch.empty((H, W, cout), dtype=torch.bfloat16, device="cuda")
    L = binding.lib()
    check(L.cgh_net_conv3x3(P(x1), c1, int(up), P(x2), c2, H, W, P(w), P(b), cout,
                            int(case["relu"]), P(out32), P(out16), stream()))
    xin = U.conv_input(x1n, x2n, up)
    ref = U.conv3x3(xin, wn, b.cpu().numpy())
    torch.cuda.synchronize()
    e = rel(out32.cpu().numpy(), ref)
    say("forward rel", e)
    assert e <= TOL
    r16 = U.bf16(U.relu(ref) if case["relu"] else ref)
    g16 = out16.to(torch.float64).cpu().numpy()
    # BF16 of the FP32 sum equals BF16 of the FP64 sum except at near-ties
    assert np.mean(g16 != r16) < 1e-3
    assert np.all(np.abs(g16 - r16) <= 2.0 ** -7 * np.abs(r16) + 1e-5 * np.abs(ref).max())
    # input adjoint through the flipped weights (the convolution needs cin % 32 == 0)
    gy, gyn = bf((H, W, cout), rng)
    gx_ref, gw_ref, gb_ref = U.conv3x3_backward(xin, wn, gyn)
    if cin % 32 == 0:
        wt = torch.empty((cin, 3, 3, cout), dtype=torch.bfloat16, device="cuda")
        check(L.cgh_net_flip_weights(P(w), cout, cin, P(wt), stream()))
        gx = torch.empty((H, W, cin), dtype=torch.float32, device="cuda")
        check(L.cgh_net_conv3x3(P(gy), cout, 0, None, 0, H, W, P(wt), None, cin, 0, P(gx), None,
                                stream()))
        torch.cuda.synchronize()
        e = rel(gx.cpu().numpy(), gx_ref)
        say("input adjoint rel", e)
        assert e <= TOL
        if up:
            # the upsampled part goes back to half resolution, the skip part stays
            g1 = torch.empty((h1, w1, c1), dtype=torch.float32, device="cuda")
            check(L.cgh_net_up_adjoint(P(gx), H, W, cin, c1, P(g1), stream()))
            torch.cuda.synchronize()
            assert rel(g1.cpu().numpy(), U.up2_adjoint(gx_ref[:, :, :c1])) <= TOL
    # weight and bias gradients
    ws = L.cgh_net_wgrad_workspace(H, W, cin, cout)
    scratch = torch.empty(ws // 4 + 4, dtype=torch.float32, device="cuda")
    gw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device="cuda")
    gb = torch.empty(cout, dtype=torch.float32, device="cuda")
    check(L.cgh_net_conv3x3_wgrad(P(x1), c1, int(up), P(x2), c2, H, W, P(gy), cout, P(gw), P(gb),
                                  P(scratch), ws, stream()))
    torch.cuda.synchronize()
    ew, eb = rel(gw.cpu().numpy(), gw_ref), rel(gb.cpu().numpy(), gb_ref)
    say("weight / bias gradient rel", ew, eb)
    assert ew <= TOL and eb <= TOL


def test_wgrad_many_splits_is_deterministic():
    """128 x 96 pixels: many splits of the pixel range (256 ranges of three
    16-pixel row chunks); two runs bitwise equal."""
    rng = np.random.default_rng(3)
    H, W, c1, cout = 128, 96, 32, 64
    x1, x1n = bf((H, W, c1), rng)
    gy, gyn = bf((H, W, cout), rng)
    L = binding.lib()
    ws = L.cgh_net_wgrad_workspace(H, W, c1, cout)
    scratch = torch.empty(ws // 4 + 4, dtype=torch.float32, device="cuda")
    outs = []
    for _ in range(2):
        gw = torch.empty((cout, 3, 3, c1), dtype=torch.float32, device="cuda")
        gb = torch.empty(cout, dtype=torch.float32, device="cuda")
        check(L.cgh_net_conv3x3_wgrad(P(x1), c1, 0, None, 0, H, W, P(gy), cout, P(gw), P(gb),
                                      P(scratch), ws, stream()))
        torch.cuda.synchronize()
        outs.append((gw.cpu().numpy(), gb.cpu().numpy()))
    _, gw_ref, gb_ref = U.conv3x3_backward(x1n, np.zeros((cout, 3, 3, c1)), gyn)
    assert rel(outs[0][0], gw_ref) <= TOL and rel(outs[0][1], gb_ref) <= TOL
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_glue_kernels():
    rng = np.random.default_rng(4)
    L = binding.lib()
    H, W, C = 10, 14, 24
    x, xn = bf((H, W, C), rng)
    p = torch.empty((H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    check(L.cgh_net_pool2(P(x), H, W, C, P(p), stream()))
    g = torch.from_numpy(rng.standard_normal((H, W, 40)).astype(np.float32)).cuda()
    up = torch.empty((H // 2, W // 2, C), dtype=torch.float32, device="cuda")
    check(L.cgh_net_up_adjoint(P(g), H, W, 40, C, P(up), stream()))
    gp = torch.from_numpy(rng.standard_normal((H // 2, W // 2, C)).astype(np.float32)).cuda()
    comb = torch.empty((H, W, C), dtype=torch.float32, device="cuda")
    check(L.cgh_net_grad_combine(P(gp), P(g), 40, 16, H, W, C, P(comb), stream()))
    a, an = bf((H, W, C), rng)
    gf = torch.from_numpy(rng.standard_normal((H, W, C)).astype(np.float32)).cuda()
    rg = torch.empty((H, W, C), dtype=torch.bfloat16, device="cuda")
    check(L.cgh_net_relu_grad(P(gf), P(a), H * W * C, P(rg), stream()))
    cast = torch.empty((H, W, C), dtype=torch.bfloat16, device="cuda")
    check(L.cgh_net_cast_bf16(P(gf), H * W * C, P(cast), stream()))
    torch.cuda.synchronize()
    # BF16 of an FP32 four-term sum against BF16 of the exact mean: equal but
    # for rare near-ties, and then one BF16 ulp apart
    pg, pr = p.to(torch.float64).cpu().numpy(), U.bf16(U.pool2(xn))
    assert np.mean(pg != pr) < 1e-3
    assert np.all(np.abs(pg - pr) <= 2.0 ** -7 * np.abs(pr) + 1e-30)
    gn = g.cpu().numpy().astype(np.float64)
    assert rel(up.cpu().numpy(), U.up2_adjoint(gn[:, :, :C])) <= 1e-7
    assert rel(comb.cpu().numpy(), U.pool2_adjoint(gp.cpu().numpy().astype(np.float64))
               + gn[:, :, 16:16 + C]) <= 1e-7
    gfn = gf.cpu().numpy().astype(np.float64)
    assert np.array_equal(rg.to(torch.float64).cpu().numpy(), U.bf16(gfn * (an > 0)))
    assert np.array_equal(cast.to(torch.float64).cpu().numpy(), U.bf16(gfn))
    # torch's own round to nearest even agrees on the cast
    assert torch.equal(cast.cpu(), gf.cpu().to(torch.bfloat16))


@pytest.mark.parametrize("C", [1, 3])
def test_lattice_gather_and_scatter(C):
    rng = np.random.default_rng(5)
    H, W, gy, gx = 64, 96, 29, 43
    out = (0.4 * rng.standard_normal((H, W, 8 * C))).astype(np.float32)
    out[::7, ::5, 0] = 200.0   # some means pushed past the canvas: the clip
    n = gy * gx
    L = binding.lib()
    net = torch.from_numpy(out).cuda()
    params = torch.empty((6 + 2 * C) * n, dtype=torch.float32, device="cuda")
    check(L.cgh_net_lattice_gather(P(net), H, W, gy, gx, C, P(params), stream()))
    g = torch.from_numpy(rng.standard_normal((6 + 2 * C) * n).astype(np.float32)).cuda()
    gnet = torch.full((H, W, 8 * C), 7.0, dtype=torch.float32, device="cuda")
    check(L.cgh_net_lattice_scatter(P(net), P(g), H, W, gy, gx, C, P(gnet), stream()))
    torch.cuda.synchronize()
    ref = U.gather(out, H, W, gy, gx, C)
    got = binding.unpack(params.cpu(), n, C)
    for k in binding.PARAM_KEYS:
        assert rel(got[k].numpy(), np.asarray(ref[k]).reshape(got[k].shape)) <= 1e-7, k
    gd = binding.unpack(g.cpu(), n, C)
    gref = U.gather_adjoint({k: gd[k].numpy().astype(np.float64) for k in gd}, out, H, W, gy, gx,
                            C)
    assert rel(gnet.cpu().numpy(), gref) <= 1e-7


# ---------------------------------------------------------------------------
# The whole network and the learned initialiser against the oracle.  Every
# activation is stored in BF16, and where an FP32 sum and the FP64 sum of the
# same terms fall on either side of a BF16 rounding tie the two stored values
# differ by one BF16 ulp (2^-7 relative); that happens to ~0.1 % of the
# elements of a layer and compounds over the 15 layers.  So the wiring is
# checked layer by layer on the GPU's own inputs (exact up to those flips),
# the weight gradients on the GPU's own activations, and the end-to-end output
# against the fully independent oracle run at a bar that allows the
# compounding (2e-2 relative L2).
# ---------------------------------------------------------------------------
LAYER_FLIPS = 2e-3
GRAD_TOL_NET = 5e-3
E2E_TOL = 2e-2


def gpu_cache(net, x16):
    """The oracle's cache built from the GPU's stored activations: the exact
    inputs each GPU convolution read, and its stored output for the ReLU test."""
    A = {k: v.to(torch.float64).cpu().numpy() for k, v in net.act.items()}
    Pl = {k: v.to(torch.float64).cpu().numpy() for k, v in net.pooled.items()}
    x = x16.to(torch.float64).cpu().numpy()
    nl = len(net.widths)
    cache = {"in": {}, "pre": {}}
    for l in range(nl):
        cache["in"][f"enc{l}a"] = (x if l == 0 else Pl[l - 1], None, False)
        cache["in"][f"enc{l}b"] = (A[f"enc{l}a"], None, False)
    for l in range(nl - 2, -1, -1):
        below = A[f"dec{l + 1}b"] if l + 1 < nl - 1 else A[f"enc{nl - 1}b"]
        cache["in"][f"dec{l}a"] = (below, A[f"enc{l}b"], True)
        cache["in"][f"dec{l}b"] = (A[f"dec{l}a"], None, False)
    cache["in"]["head"] = (A["dec0b"], None, False)
    for k, v in A.items():
        cache["pre"][k] = v
    return cache, A, Pl


def test_unet_forward_backward_matches_oracle():
    from paper_2511_15022_amd import learned_init as LI
    H, W = 32, 48
    say("unet", H, W)
    rng = np.random.default_rng(21)
    net = LI.UNet(H, W, seed=22)
    wd = net.get_weights()
    for k in wd:  # nonzero biases exercise the bias path
        if k.endswith(".b"):
            wd[k] = (0.05 * rng.standard_normal(wd[k].shape)).astype(np.float32)
    net.set_weights(wd)
    x16, xn = bf((H, W, 8), rng)
    out = net.forward(x16).clone()
    g = (rng.standard_normal((H, W, 8))).astype(np.float32)
    net.backward(torch.from_numpy(g).cuda(), x16)
    torch.cuda.synchronize()
    cache, A, Pl = gpu_cache(net, x16)
    # 1. layer by layer on the GPU's own inputs
    for name, cu, cs, co, relu in net.layers:
        h, skip, up = cache["in"][name]
        z = U.conv3x3(U.conv_input(h, skip, up), U.bf16(wd[name]), wd[name + ".b"])
        if name == "head":
            e = rel(out.cpu().numpy(), z)
            assert e <= TOL, (name, e)
            continue
        ref16, got = U.bf16(U.relu(z)), A[name]
        frac = np.mean(ref16 != got)
        assert frac <= LAYER_FLIPS, (name, frac)
        assert np.all(np.abs(ref16 - got) <= 2.0 ** -7 * np.abs(ref16) + 1e-6 * np.abs(z).max()), name
    for l, p in Pl.items():
        src = A[f"enc{l}b"]
        pr = U.bf16(U.pool2(src))
        assert np.mean(pr != p) <= LAYER_FLIPS
    # 2. weight gradients on the GPU's activations
    arch = U.architecture()
    grads = U.backward(arch, wd, cache, g.astype(np.float64))
    host = net.grad.cpu().numpy()
    worst = (0.0, "")
    for name, cu, cs, co, _ in net.layers:
        o, n = net.off[name]
        worst = max(worst, (rel(host[o:o + n].reshape(co, 3, 3, cu + cs), grads[name]), name))
        o, n = net.off[name + ".b"]
        worst = max(worst, (rel(host[o:o + n], grads[name + ".b"]), name + ".b"))
    say("worst gradient rel (GPU activations)", worst)
    assert worst[0] <= GRAD_TOL_NET
    # 3. end to end against the independent oracle run
    ref, _ = U.forward(arch, wd, xn)
    e = rel(out.cpu().numpy(), ref)
    say("end-to-end output rel", e)
    assert e <= E2E_TOL


@pytest.mark.parametrize("lams", [[515e-9], [639e-9, 515e-9, 473e-9]])
def test_initializer_prediction_and_training_gradients(lams):
    """Features (the library's back-propagation of sqrt(T)), network, lattice
    gather, rendering, MSE backward, scatter and network backward, against the
    oracle's composition of the same steps; one and three colour channels."""
    from oracle import oracle as O
    from paper_2511_15022_amd import learned_init as LI, synth
    H, W, pitch, z = 32, 48, 8e-6, 2e-3
    C = len(lams)
    say("initializer", C)
    init = LI.Initializer(H, W, pitch, lams, z, pad=(64, 96), seed=31)
    T = synth.target(32, C, H, W)[0]
    Tg = torch.from_numpy(T).cuda()
    params = init.predict(Tg).clone()
    x16 = init.x16.clone()
    torch.cuda.synchronize()
    # the oracle's features: sqrt(T) propagated by -z, rounded to BF16
    back = O.propagate(np.sqrt(np.maximum(T, 0)).astype(np.complex128),
                       O.Optics(H, W, C, 64, 96, pitch, lams, [-z]))[0]
    feats = np.zeros((H, W, 8 * C))
    for c in range(C):
        feats[..., 8 * c], feats[..., 8 * c + 1] = T[c], np.sqrt(np.maximum(T[c], 0))
        feats[..., 8 * c + 2], feats[..., 8 * c + 3] = back[c].real, back[c].imag
        feats[..., 8 * c + 4] = np.abs(back[c])
    fr = U.bf16(feats)
    fg = x16.to(torch.float64).cpu().numpy()
    # BF16 of the FP32 and FP64 back-propagations: equal but for near-ties
    assert np.mean(fg != fr) < 2e-3 and rel(fg, fr) < 2e-3
    wd = init.net.get_weights()
    arch = U.architecture(c_in=8 * C, c_out=8 * C)
    out = init.net.out.cpu().numpy().astype(np.float64)
    cache, _, _ = gpu_cache(init.net, x16)
    # the lattice gather of the GPU's network output is exact up to FP32 rounding
    ref = U.gather(out, H, W, init.gy, init.gx, C)
    got = binding.unpack(params.cpu(), init.n, C)
    for k in binding.PARAM_KEYS:
        e = rel(got[k].numpy(), np.asarray(ref[k]).reshape(got[k].shape))
        assert e <= 1e-6, (k, e)
    # one training step: gradients of the network's weights
    init.train_step(Tg, lr=0.0)
    torch.cuda.synchronize()
    opt = O.Optics(H, W, C, 64, 96, pitch, lams, [z])
    p32 = {k: np.asarray(got[k].numpy(), np.float32) for k in got}
    fb = O.forward_backward(p32, T[None], opt)
    g_out = U.gather_adjoint({k: np.asarray(v, np.float64) for k, v in fb["grads"].items()},
                             out, H, W, init.gy, init.gx, C)
    grads = U.backward(arch, wd, cache, g_out)
    host = init.net.grad.cpu().numpy()
    worst = 0.0
    for name, cu, cs, co, _ in init.net.layers:
        o, n = init.net.off[name]
        worst = max(worst, rel(host[o:o + n].reshape(co, 3, 3, cu + cs), grads[name]))
    say("initializer: worst weight-gradient rel", worst, "loss", init.loss.cpu().numpy(),
        fb["loss"])
    assert abs(init.loss.cpu().numpy()[0] - fb["loss"]) <= 1e-4 * fb["loss"]
    assert worst <= GRAD_TOL_NET


def test_trained_initializer_beats_the_grid_initialisation():
    """What the trained network gains over the method without it: after a
    short training (200 steps on 16 seeded 64 x 64 RGB targets), its prediction
    for held-out targets renders far closer to them than the plain lattice
    (zero network output) does, and stays ahead after 50 optimiser steps."""
    from paper_2511_15022_amd import learned_init as LI, synth
    H = W = 64
    lams, z = [639e-9, 515e-9, 473e-9], 5e-3
    init = LI.Initializer(H, W, 8e-6, lams, z, seed=0)
    LI.scale_head(init, 0.01)
    pool = [torch.from_numpy(synth.target(1000 + i, 3, H, W)[0]).cuda() for i in range(16)]
    log, secs = LI.train(init, pool, 200, 3e-4)
    say("training psnr first/last", log[:10, 1].mean(), log[-10:, 1].mean(), "seconds", secs)
    gains0, gains50 = [], []
    for i in range(3):
        T = torch.from_numpy(synth.target(9000 + i, 3, H, W)[0]).cuda()
        pl, tl = LI.optimise(init.ctx, init.predict(T).clone(), init.n, T, 51)
        pg, tg = LI.optimise(init.ctx, init.grid(), init.n, T, 51)
        gains0.append(pl[0] - pg[0])
        gains50.append(pl[50] - pg[50])
    say("PSNR gain over the grid init at step 0 / 50:", gains0, gains50)
    assert min(gains0) > 10.0
    assert min(gains50) > 3.0
