"""GPU tests of the serving path: cgh_set_optics, the graph-captured solve
(cgh_solve_*) and the stream scheduler (paper_2511_15022_amd/serve.py), all
through the C ABI.  The graph and the scheduler are checked bit for bit
against the same calls made one by one (whose kernels the oracle parity tests
cover); the optics update and the FFT plans of the serving sizes (pads 1024^2,
1536 x 2048, 2048^2, 4096^2) are checked against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from paper_2511_15022_amd import binding, serve, synth

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


def test_set_optics_matches_a_fresh_context(O):
    """Transfer tables after cgh_set_optics equal, bit for bit, those of a
    context created with the new optics; propagation then matches the oracle.
    The 1080 x 1920 class also keeps a column-major copy of the table."""
    for H, W, Hp, Wp in ((40, 56, 80, 120), (1080, 1920, 2160, 3840)):
        say("set_optics", H, W)
        lams, zs = [639e-9, 473e-9], [2e-3, -4e-3]
        new_l, new_z = [515e-9, 700e-9], [7.5e-3, 3e-3]
        a = binding.Context(H, W, 2, 8e-6, lams, zs, pad=(Hp, Wp), max_gaussians=1)
        a.set_optics(new_l, new_z)
        b = binding.Context(H, W, 2, 8e-6, new_l, new_z, pad=(Hp, Wp), max_gaussians=1)
        for ch in range(2):
            for l in range(2):
                assert torch.equal(a.get_transfer(ch, l), b.get_transfer(ch, l))
        rng = np.random.default_rng(11)
        f = (rng.standard_normal((2, H, W)) + 1j * rng.standard_normal((2, H, W))).astype(np.complex64)
        tf = torch.from_numpy(f).cuda()
        _, ua = a.propagate(tf, intensity=False, field_out=True)
        _, ub = b.propagate(tf, intensity=False, field_out=True)
        assert torch.equal(ua, ub)
        if H < 100:
            ref = O.propagate(f.astype(np.complex128), O.Optics(H, W, 2, Hp, Wp, 8e-6, new_l, new_z))
            assert rel_l2(ua.cpu().numpy(), ref) <= FIELD_TOL


def test_set_optics_rejects_bad_values():
    ctx = binding.Context(16, 16, 1, 8e-6, [515e-9], [2e-3], max_gaussians=1)
    before = ctx.get_transfer().clone()
    for lam, z in (([0.0], [1e-3]), ([float("nan")], [1e-3]), ([515e-9], [float("inf")])):
        with pytest.raises(binding.CghError):
            ctx.set_optics(lam, z)
    assert torch.equal(ctx.get_transfer(), before)


def _eager(ctx, P, n, T, steps, lr):
    log = serve.solve_eager(ctx, P, n, T, steps, lr)
    torch.cuda.synchronize()
    return log


def test_solve_graph_matches_eager_steps(O):
    """Two launches of a captured 6-step solve (three colours, two planes),
    the second from new parameters: every launch equals the eager calls bit
    for bit (parameters and loss log), so the graph restarts the moments; the
    first logged loss matches the oracle."""
    H, W, C, n, steps, lr = 48, 80, 3, 500, 6, 2e-3
    lams, zs = [639e-9, 515e-9, 473e-9], [4e-3, 6e-3]
    T = torch.from_numpy(synth.target(121, C, H, W, L=2)).cuda()
    ctx = binding.Context(H, W, C, 8e-6, lams, zs, pad=(90, 160), max_gaussians=n)
    P = torch.empty(binding.param_count(n, C), dtype=torch.float32, device="cuda")
    solve = binding.Solve(ctx, P, n, T, steps, lr=lr)
    ref_ctx = binding.Context(H, W, C, 8e-6, lams, zs, pad=(90, 160), max_gaussians=n)
    for rep, seed in enumerate((122, 123)):
        p = synth.params(seed, n, H, W, C)
        P.copy_(binding.pack(p, device="cuda"))
        torch.cuda.synchronize()
        solve.launch()
        torch.cuda.synchronize()
        Pe = binding.pack(p, device="cuda")
        log = _eager(ref_ctx, Pe, n, T, steps, lr)
        say("solve launch", rep, "loss", solve.loss_log[0, 0].item(), solve.loss_log[-1, 0].item())
        assert torch.equal(P, Pe)
        assert torch.equal(solve.loss_log, log)
        assert solve.loss_log[-1, 0].item() < solve.loss_log[0, 0].item()
        if rep == 0:
            opt = O.Optics(H, W, C, 90, 160, 8e-6, lams, zs)
            ref = O.forward(p, T.cpu().numpy(), opt)["loss"]
            assert abs(solve.loss_log[0, 0].item() - ref) <= 1e-4 * ref
    solve.close()


def test_solve_create_rejections():
    ctx = binding.Context(16, 16, 1, 8e-6, [515e-9], [2e-3], max_gaussians=10)
    P = torch.zeros(binding.param_count(10, 1), device="cuda")
    T = torch.zeros((1, 1, 16, 16), device="cuda")
    for kw in (dict(steps=0), dict(steps=10001), dict(lr=float("nan"))):
        args = dict(steps=3, lr=1e-3)
        args.update(kw)
        with pytest.raises(binding.CghError) as e:
            binding.Solve(ctx, P, 10, T, args["steps"], lr=args["lr"])
        assert e.value.status == 1
    ctx.profile_begin("raster")
    with pytest.raises(binding.CghError) as e:
        binding.Solve(ctx, P, 10, T, 3)
    assert e.value.status == 6
    ctx.profile_end()
    s = binding.Solve(ctx, P, 10, T, 3)  # capture works again once timing stops
    s.close()


def test_server_matches_standalone_solves():
    """Seven requests of three sizes with their own optics on two streams:
    every result (parameters and loss log) equals the eager solve of that
    request on a context created with its optics, bit for bit."""
    sizes = ((40, 60), (48, 64), (32, 32))
    reqs = serve.make_requests(7, seed=131, sizes=sizes)
    steps, lr = 5, 1e-3
    server = serve.Server(steps, lr=lr, max_streams=2)
    res = server.run(reqs, streams=2)
    assert len(res["latency_ms"]) == 7 and set(res["stream_of"].values()) == {0, 1}
    for r in reqs:
        ctx = binding.Context(r.H, r.W, 1, serve.PITCH, [r.wavelength], [r.z], max_gaussians=r.n)
        P = r.params.clone()
        log = _eager(ctx, P, r.n, r.target, steps, lr)
        say("request", r.index, r.H, r.W, r.wavelength, round(r.z, 5))
        assert torch.equal(r.out_params, P)
        assert torch.equal(r.out_loss, log)
    # a second run reuses the slots and graphs and gives the same results
    first = [r.out_params.clone() for r in reqs]
    server.run(reqs, streams=1)
    for r, f in zip(reqs, first):
        assert torch.equal(r.out_params, f)


def test_batch_server_matches_standalone_solves():
    """Nine requests of three sizes served as batched solves (at most two
    holograms per batch, so a class spans several batches and batch sizes),
    after the tile-shape autotuner has chosen each class's tile: every result
    equals the eager solve of that request alone on a context with its optics
    and the chosen tile, bit for bit."""
    sizes = ((40, 60), (48, 64), (32, 32))
    reqs = serve.make_requests(9, seed=151, sizes=sizes)
    steps, lr = 5, 1e-3
    server = serve.BatchServer(steps, lr=lr, max_streams=2, max_batch=2)
    timings = server.tune_tiles(reqs, probe_steps=3)
    assert set(timings) == {(r.H, r.W) for r in reqs}
    for key, t in timings.items():
        say("tile timings", key, t, "chosen", server.tile_of(*key))
        assert set(t) == set(binding.TILE_SHAPES) and server.tile_of(*key) in t
    res = server.run(reqs, streams=2)
    assert len(res["latency_ms"]) == 9
    assert max(b for _, _, b in res["batches"]) == 2
    for r in reqs:
        ctx = binding.Context(r.H, r.W, 1, serve.PITCH, [r.wavelength], [r.z], max_gaussians=r.n,
                              tile=server.tile_of(r.H, r.W))
        P = r.params.clone()
        log = _eager(ctx, P, r.n, r.target, steps, lr)
        say("batched request", r.index, r.H, r.W)
        assert torch.equal(r.out_params, P)
        assert torch.equal(r.out_loss, log)


def test_mixed_server_matches_standalone_solves():
    """Eight requests of three sizes served by the mixed server with two
    classes batched (at most two holograms per batch) and one class one
    hologram at a time, on two shared streams: every result equals the eager
    solve of that request alone on a context with its optics (and, for a
    batched class, its batch's tile), bit for bit."""
    sizes = ((40, 60), (48, 64), (32, 32))
    reqs = serve.make_requests(8, seed=171, sizes=sizes)
    steps, lr = 5, 1e-3
    streams = [torch.cuda.Stream() for _ in range(2)]
    bserver = serve.BatchServer(steps, lr=lr, max_batch=2, streams=streams)
    bserver.tiles[(48, 64)] = (32, 8)
    sserver = serve.Server(steps, lr=lr, streams=streams)
    # made-up costs that batch (40, 60) and (48, 64) and keep (32, 32) single
    batch_ms = {(40, 60): (1.0, 2), (48, 64): (1.0, 2), (32, 32): (4.0, 2)}
    single_ms = {(40, 60): 1.0, (48, 64): 1.0, (32, 32): 1.0}
    mixed = serve.MixedServer(bserver, sserver, batch_ms, single_ms)
    assert mixed.batched == {(40, 60), (48, 64)}
    res = mixed.run(reqs, streams=2)
    assert len(res["latency_ms"]) == 8 and set(res["stream_of"].values()) <= {0, 1}
    for r in reqs:
        tile = bserver.tile_of(r.H, r.W) if (r.H, r.W) in mixed.batched else (16, 16)
        ctx = binding.Context(r.H, r.W, 1, serve.PITCH, [r.wavelength], [r.z], max_gaussians=r.n,
                              tile=tile)
        P = r.params.clone()
        log = _eager(ctx, P, r.n, r.target, steps, lr)
        say("mixed request", r.index, r.H, r.W, tile)
        assert torch.equal(r.out_params, P)
        assert torch.equal(r.out_loss, log)


@pytest.mark.parametrize("H,W", [(512, 512), (768, 1024)])
def test_serving_sizes_forward_backward_match_oracle(O, H, W):
    """Full-size serving classes (pads 1024^2 and 1536 x 2048, the runtime
    FFT plans) through rasterize + backward against the oracle, with 1500
    Gaussians (the oracle's brute-force sum bounds n)."""
    n, lam, z = 1500, 473e-9, 7.3e-3
    say("serving size", H, W)
    p = synth.params(141, n, H, W, 1)
    T = synth.target(142, 1, H, W)
    ctx = binding.Context(H, W, 1, 8e-6, [lam], [z], max_gaussians=n)
    P = binding.pack(p, device="cuda")
    field = ctx.rasterize(P, n)
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    gfield = torch.empty_like(field)
    grads = ctx.backward(P, n, field, torch.from_numpy(T).cuda(), loss=loss, grad_field=gfield)
    torch.cuda.synchronize()
    opt = O.Optics(H, W, 1, 2 * H, 2 * W, 8e-6, [lam], [z])
    ref = O.forward_backward(p, T, opt)
    mask, _ = O.ambiguous_mask(p, opt, AMBIGUOUS_BAND)
    assert mask.sum() <= max(3, 1e-3 * mask.size)
    assert rel_l2(field.cpu().numpy(), ref["field"], mask) <= FIELD_TOL
    assert abs(loss[0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    assert rel_l2(gfield.cpu().numpy(), ref["grad_field"]) <= GRAD_TOL
    views = binding.unpack(grads.cpu(), n, 1)
    for k in binding.PARAM_KEYS:
        e = rel_l2(views[k].numpy(), ref["grads"][k])
        assert e <= GRAD_TOL, (k, e)


@pytest.mark.parametrize("H,W", [(1024, 1024), (2048, 2048)])
def test_serving_sizes_propagation_match_oracle(O, H, W):
    """Propagation and its adjoint at the square serving classes (pads 2048^2
    and 4096^2) against the oracle."""
    say("serving propagate", H, W)
    rng = np.random.default_rng(151)
    f = (rng.standard_normal((1, H, W)) + 1j * rng.standard_normal((1, H, W))).astype(np.complex64)
    g = rng.standard_normal((1, 1, H, W)).astype(np.float32)
    ctx = binding.Context(H, W, 1, 8e-6, [639e-9], [9.1e-3], max_gaussians=1)
    tf = torch.from_numpy(f).cuda()
    _, u = ctx.propagate(tf, intensity=False, field_out=True)
    gf = ctx.propagate_adjoint(tf, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    opt = O.Optics(H, W, 1, 2 * H, 2 * W, 8e-6, [639e-9], [9.1e-3])
    f64 = f.astype(np.complex128)
    u_ref = O.propagate(f64, opt)
    assert rel_l2(u.cpu().numpy(), u_ref) <= FIELD_TOL
    # dL/dI = g  =>  dL/du = 2 g u, then the adjoint propagation
    gf_ref = O.propagate_adjoint(2.0 * g.astype(np.float64) * u_ref, opt)
    assert rel_l2(gf.cpu().numpy(), gf_ref) <= FIELD_TOL


@pytest.mark.parametrize("case", [
    # quarter rows M = 512 (W < 2M), four-chain columns M = 384 (H < 2M), 2 colours x 2 planes
    dict(H=700, W=900, Hp=1536, Wp=2048, C=2, zs=[3e-3, -6e-3]),
    # quarter rows M = 256, four-chain columns M = 256
    dict(H=300, W=500, Hp=1024, Wp=1024, C=1, zs=[4e-3]),
    # four-chain columns M = 256 with an odd number of column tiles (15), runtime rows
    dict(H=400, W=60, Hp=1024, Wp=120, C=2, zs=[2e-3]),
])
def test_four_chain_pads_ragged_match_oracle(O, case):
    """The quarter-length row passes and four-chain column passes at the
    serving pads with ragged H, W (fewer rows/columns than half the pad),
    several colours and planes: propagation, its adjoint and a fused
    forward + backward with Gaussians against the oracle."""
    say("four-chain pads", case)
    H, W, Hp, Wp, C, zs = (case[k] for k in ("H", "W", "Hp", "Wp", "C", "zs"))
    lams = [639e-9, 473e-9][:C]
    L = len(zs)
    rng = np.random.default_rng(161)
    f = (rng.standard_normal((C, H, W)) + 1j * rng.standard_normal((C, H, W))).astype(np.complex64)
    gI = rng.standard_normal((L, C, H, W)).astype(np.float32)
    n = 600
    ctx = binding.Context(H, W, C, 8e-6, lams, zs, pad=(Hp, Wp), max_gaussians=n)
    opt = O.Optics(H, W, C, Hp, Wp, 8e-6, lams, zs)
    tf = torch.from_numpy(f).cuda()
    _, u = ctx.propagate(tf, intensity=False, field_out=True)
    g = ctx.propagate_adjoint(tf, torch.from_numpy(gI).cuda())
    torch.cuda.synchronize()
    u_ref = O.propagate(f.astype(np.complex128), opt)
    assert rel_l2(u.cpu().numpy(), u_ref) <= FIELD_TOL
    g_ref = O.propagate_adjoint(2.0 * gI.astype(np.float64) * u_ref, opt)
    assert rel_l2(g.cpu().numpy(), g_ref) <= FIELD_TOL
    p = synth.params(162, n, H, W, C)
    T = synth.target(163, C, H, W, L=L)
    P = binding.pack(p, device="cuda")
    field = ctx.rasterize(P, n)
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    gfield = torch.empty_like(field)
    grads = ctx.backward(P, n, field, torch.from_numpy(T).cuda(), loss=loss, grad_field=gfield)
    torch.cuda.synchronize()
    ref = O.forward_backward(p, T, opt)
    assert abs(loss[0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    assert rel_l2(gfield.cpu().numpy(), ref["grad_field"]) <= GRAD_TOL
    views = binding.unpack(grads.cpu(), n, C)
    for k in binding.PARAM_KEYS:
        e = rel_l2(views[k].numpy(), ref["grads"][k])
        assert e <= GRAD_TOL, (k, e)
