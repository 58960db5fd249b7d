"""GPU tests of the tile shapes, batched contexts (several holograms of one
size in every launch), the non-finite check and the solve graph over a batch,
all through the C ABI.

* Tile shapes (16 x 16, 32 x 8, 16 x 8, 8 x 8): each shape matches the FP64
  oracle (field 1e-4, gradients 1e-3 per group), and the shapes agree with
  each other to FP32 rounding: the pixel offsets from a Gaussian's mean are
  formed from the tile origin (as in the adjoint, so that forward and adjoint
  take the same support decisions), which changes their last bits with the
  tile shape; pixels of pairs within the rounding band of the support
  boundary are left out of the field comparison.
* Batches: hologram b of a batched context gives, bit for bit, what a single
  context with that hologram's parameters, target and optics gives (the same
  kernels over the same tile lists), and one hologram is checked against the
  oracle."""
import sys

import numpy as np
import pytest
import torch

from paper_2511_15022_amd import binding, synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-4
GRAD_TOL = 1e-3
AMBIGUOUS_BAND = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, mask=None):
    a, b = np.asarray(a), np.asarray(b)
    if mask is not None:
        a, b = a[..., ~mask], b[..., ~mask]
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def group_errors(g_gpu, g_ref, n, C):
    views = binding.unpack(torch.as_tensor(g_gpu), n, C)
    return {k: rel_l2(views[k].numpy(), g_ref[k]) for k in binding.PARAM_KEYS}


@pytest.mark.parametrize("case", [
    dict(H=256, W=256, C=1, n=4096, lambdas=[515e-9], zs=[2e-3]),
    dict(H=100, W=135, C=3, n=900, lambdas=[639e-9, 515e-9, 473e-9], zs=[4e-3, 6e-3]),
])
def test_tile_shapes_match_oracle_and_each_other(O, case):
    H, W, C, n, zs = case["H"], case["W"], case["C"], case["n"], case["zs"]
    L = len(zs)
    p = synth.params(201, n, H, W, C)
    T = synth.target(202, C, H, W, L=L)
    opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, case["lambdas"], zs)
    ref = O.forward_backward(p, T, opt)
    mask, _ = O.ambiguous_mask(p, opt, AMBIGUOUS_BAND)
    assert mask.sum() <= max(3, 1e-3 * mask.size)
    P = binding.pack(p, device="cuda")
    Tt = torch.from_numpy(T).cuda()
    base_field = base_grads = None
    for tile in binding.TILE_SHAPES:
        say("tile", tile, case)
        ctx = binding.Context(H, W, C, 8e-6, case["lambdas"], zs, max_gaussians=n, tile=tile)
        field = ctx.rasterize(P, n).clone()
        loss = torch.zeros(2, dtype=torch.float64, device="cuda")
        grads = ctx.backward(P, n, field, Tt, loss=loss).clone()
        _, ok = ctx.read_status()
        assert ok
        assert rel_l2(field.cpu().numpy(), ref["field"], mask) <= FIELD_TOL
        assert abs(loss[0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
        errs = group_errors(grads.cpu(), ref["grads"], n, C)
        say("grad vs oracle", errs)
        for k, e in errs.items():
            assert e <= GRAD_TOL, (tile, k, e)
        if base_field is None:
            base_field, base_grads = field, grads
        else:
            e = rel_l2(field.cpu().numpy(), base_field.cpu().numpy(), mask)
            say("field vs 16 x 16", e)
            assert e <= 1e-6, (tile, e)
            g = binding.unpack(grads.cpu(), n, C)
            b = binding.unpack(base_grads.cpu(), n, C)
            for k in binding.PARAM_KEYS:
                e = rel_l2(g[k].numpy(), b[k].numpy())
                assert e <= 1e-5, (tile, k, e)


def batch_case(B, H, W, C, n, L, seed):
    rng = np.random.default_rng(seed)
    lams = [[float(rng.choice([639e-9, 515e-9, 473e-9])) for _ in range(C)] for _ in range(B)]
    zs = [[float(rng.uniform(2e-3, 8e-3)) for _ in range(L)] for _ in range(B)]
    ps = [synth.params(seed + 1 + b, n, H, W, C) for b in range(B)]
    Ts = [synth.target(seed + 20 + b, C, H, W, L=L) for b in range(B)]
    return lams, zs, ps, Ts


def stack_planes(arrs):
    """[B] arrays of [L][C][H][W] -> [L][B][C][H][W]"""
    return np.ascontiguousarray(np.stack(arrs, axis=1))


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_batch_matches_single_contexts(O, tile):
    B, H, W, C, n, L = 3, 48, 80, 2, 300, 2
    say("batch", B, H, W, C, n, L, tile)
    lams, zs, ps, Ts = batch_case(B, H, W, C, n, L, 300)
    bctx = binding.Context(H, W, C, 8e-6, lams[0], zs[0], pad=(90, 160), max_gaussians=n,
                           batch=B, tile=tile)
    for b in range(B):
        bctx.set_hologram_optics(b, lams[b], zs[b])
    P = torch.cat([binding.pack(p, device="cuda") for p in ps])
    T = torch.from_numpy(stack_planes(Ts)).cuda()
    field = bctx.rasterize(P, n)
    assert field.shape == (B, C, H, W)
    I, u = bctx.propagate(field, intensity=True, field_out=True)
    assert I.shape == (L, B, C, H, W)
    loss = torch.zeros(2 * B, dtype=torch.float64, device="cuda")
    gfield = torch.empty_like(field)
    grads = bctx.backward(P, n, field, T, loss=loss, grad_field=gfield)
    _, ok = bctx.read_status()
    assert ok
    per = binding.param_count(n, C)
    for b in range(B):
        ctx = binding.Context(H, W, C, 8e-6, lams[b], zs[b], pad=(90, 160), max_gaussians=n,
                              tile=tile)
        for ch in range(C):
            for l in range(L):
                assert torch.equal(bctx.get_transfer(b * C + ch, l), ctx.get_transfer(ch, l))
        Pb = binding.pack(ps[b], device="cuda")
        f1 = ctx.rasterize(Pb, n)
        assert torch.equal(field[b], f1), b
        I1, u1 = ctx.propagate(f1, intensity=True, field_out=True)
        assert torch.equal(I[:, b], I1) and torch.equal(u[:, b], u1)
        l1 = torch.zeros(2, dtype=torch.float64, device="cuda")
        g1f = torch.empty_like(f1)
        g1 = ctx.backward(Pb, n, f1, torch.from_numpy(Ts[b]).cuda(), loss=l1, grad_field=g1f)
        assert torch.equal(gfield[b], g1f), b
        assert torch.equal(grads[b * per:(b + 1) * per], g1), b
        assert abs(loss[2 * b].item() - l1[0].item()) <= 1e-12 * l1[0].item()
    # one hologram against the oracle
    b = 1
    opt = O.Optics(H, W, C, 90, 160, 8e-6, lams[b], zs[b])
    ref = O.forward_backward(ps[b], Ts[b], opt)
    mask, _ = O.ambiguous_mask(ps[b], opt, AMBIGUOUS_BAND)
    assert rel_l2(field[b].cpu().numpy(), ref["field"], mask) <= FIELD_TOL
    assert abs(loss[2 * b].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    for k, e in group_errors(grads[b * per:(b + 1) * per].cpu(), ref["grads"], n, C).items():
        assert e <= GRAD_TOL, (k, e)


def test_batch_recon_masks_and_adjoints(O):
    """L_recon with per-hologram masks ([L][B][H][W]) and the split adjoints
    over a batch, against single contexts."""
    B, H, W, C, n, L = 2, 40, 60, 1, 200, 2
    lams, zs, ps, Ts = batch_case(B, H, W, C, n, L, 400)
    Ms = [(np.random.default_rng(410 + b).uniform(0, 1, (L, H, W)) > 0.5).astype(np.float32)
          for b in range(B)]
    bctx = binding.Context(H, W, C, 8e-6, lams[0], zs[0], max_gaussians=n, batch=B)
    for b in range(B):
        bctx.set_hologram_optics(b, lams[b], zs[b])
    P = torch.cat([binding.pack(p, device="cuda") for p in ps])
    T = torch.from_numpy(stack_planes(Ts)).cuda()
    M = torch.from_numpy(np.ascontiguousarray(np.stack(Ms, axis=1))).cuda()
    field = bctx.rasterize(P, n)
    loss = torch.zeros(2 * B, dtype=torch.float64, device="cuda")
    grads = bctx.backward(P, n, field, T, loss=loss, mask=M)
    rng = np.random.default_rng(420)
    gI = torch.from_numpy(rng.standard_normal((L, B, C, H, W)).astype(np.float32)).cuda()
    gprop = bctx.propagate_adjoint(field, gI)
    gu = torch.from_numpy((rng.standard_normal((L, B, C, H, W)) +
                           1j * rng.standard_normal((L, B, C, H, W))).astype(np.complex64)).cuda()
    gfa = bctx.propagate_field_adjoint(gu)
    gr = bctx.rasterize_adjoint(P, n, gprop)
    per = binding.param_count(n, C)
    for b in range(B):
        ctx = binding.Context(H, W, C, 8e-6, lams[b], zs[b], max_gaussians=n)
        Pb = binding.pack(ps[b], device="cuda")
        f1 = ctx.rasterize(Pb, n)
        l1 = torch.zeros(2, dtype=torch.float64, device="cuda")
        g1 = ctx.backward(Pb, n, f1, torch.from_numpy(Ts[b]).cuda(), loss=l1,
                          mask=torch.from_numpy(Ms[b]).cuda())
        assert torch.equal(grads[b * per:(b + 1) * per], g1), b
        assert abs(loss[2 * b].item() - l1[0].item()) <= 1e-12 * l1[0].item()
        gp1 = ctx.propagate_adjoint(f1, gI[:, b].contiguous())
        assert torch.equal(gprop[b], gp1)
        assert torch.equal(gfa[b], ctx.propagate_field_adjoint(gu[:, b].contiguous()))
        assert torch.equal(gr[b * per:(b + 1) * per], ctx.rasterize_adjoint(Pb, n, gp1))
    opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, lams[0], zs[0])
    ref = O.forward_backward(ps[0], Ts[0], opt, mask=Ms[0])
    assert abs(loss[0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    for k, e in group_errors(grads[:per].cpu(), ref["grads"], n, C).items():
        assert e <= GRAD_TOL, (k, e)


def test_batched_solve_graph_matches_eager(O):
    """A captured solve over a batch of three holograms: two launches (the
    second from new parameters) equal the eager calls bit for bit, and each
    hologram's first logged loss matches the oracle."""
    B, H, W, C, n, steps = 3, 40, 60, 1, 250, 6
    lams, zs, ps, Ts = batch_case(B, H, W, C, n, 1, 500)
    ctx = binding.Context(H, W, C, 8e-6, lams[0], zs[0], max_gaussians=n, batch=B)
    for b in range(B):
        ctx.set_hologram_optics(b, lams[b], zs[b])
    P0 = torch.cat([binding.pack(p, device="cuda") for p in ps])
    T = torch.from_numpy(stack_planes(Ts)).cuda()
    params = P0.clone()
    solve = binding.Solve(ctx, params, n, T, steps, lr=1e-3)
    for rep in range(2):
        start = P0 if rep == 0 else P0 * 1.01
        params.copy_(start)
        torch.cuda.synchronize()
        solve.launch()
        torch.cuda.synchronize()
        # eager
        p = start.clone()
        field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device="cuda")
        g = torch.empty_like(p)
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        log = torch.zeros((steps, B, 2), dtype=torch.float64, device="cuda")
        for t in range(1, steps + 1):
            ctx.rasterize(p, n, field)
            ctx.backward(p, n, field, T, loss=log[t - 1], grads=g)
            binding.step(p, g, m, v, t, 1e-3)
        torch.cuda.synchronize()
        say("batched solve", rep, solve.loss_log[0, :, 0].tolist())
        assert torch.equal(params, p)
        assert torch.equal(solve.loss_log, log)
    for b in range(B):
        opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, lams[b], zs[b])
        q = {k: v.copy() for k, v in ps[b].items()}
        for k in q:
            q[k] = (q[k] * np.float32(1.01)).astype(np.float32)
        ref = O.forward(q, Ts[b], opt)["loss"]
        assert abs(solve.loss_log[0, b, 0].item() - ref) <= 1e-4 * ref


def test_check_finite_reports_nonfinite_values():
    """CGH_CHECK_FINITE: a NaN parameter, and an infinite target (non-finite
    loss and gradients), are reported once by cgh_read_status; clean calls
    report nothing, and an unflagged context does not check."""
    H, W, C, n = 32, 48, 2, 50
    p = synth.params(601, n, H, W, C)
    T = torch.from_numpy(synth.target(602, C, H, W)).cuda()
    ctx = binding.Context(H, W, C, 8e-6, [639e-9, 473e-9], [3e-3], max_gaussians=n,
                          check_finite=True)
    P = binding.pack(p, device="cuda")
    f = ctx.rasterize(P, n)
    ctx.backward(P, n, f, T)
    assert ctx.read_status()[1]
    bad = P.clone()
    bad[5 * n + 7] = float("nan")   # one amplitude: the geometry stays finite
    f = ctx.rasterize(bad, n)
    with pytest.raises(binding.CghError) as e:
        ctx.read_status()
    assert e.value.status == 7 and "parameters" in str(e.value)
    assert ctx.read_status()[1]      # reported once
    f = ctx.rasterize(P, n)
    Tinf = T.clone()
    Tinf[0, 0, 3, 4] = float("inf")
    ctx.backward(P, n, f, Tinf, loss=torch.zeros(2, dtype=torch.float64, device="cuda"))
    with pytest.raises(binding.CghError) as e:
        ctx.read_status()
    assert e.value.status == 7 and "loss" in str(e.value) and "gradients" in str(e.value)
    assert ctx.read_status()[1]
    plain = binding.Context(H, W, C, 8e-6, [639e-9, 473e-9], [3e-3], max_gaussians=n)
    plain.rasterize(bad, n)
    assert plain.read_status()[1]
