"""cgh_create_static (the allocation-free entry point) against cgh_create with a
caller workspace, through the C ABI: two contexts in a row on the device's
static workspace, the second smaller than the first, each giving the same
field, loss and gradients as a caller-workspace context (bit for bit: the
same kernels on the same inputs), and the first one also checked against the
FP64 oracle (field 1e-4, gradients 1e-3 per group).  Also: a configuration
too large for the static workspace and a second static context on the same
device are refused before any device work."""
import sys

import numpy as np
import pytest
import torch

from paper_2511_15022_amd import binding, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, mask=None):
    a, b = np.asarray(a), np.asarray(b)
    if mask is not None:
        a, b = a[..., ~mask], b[..., ~mask]
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


CASES = [  # the second smaller than the first
    dict(H=96, W=128, C=2, n=800, lambdas=[639e-9, 473e-9], zs=[3e-3, -2e-3], seed=701),
    dict(H=48, W=64, C=1, n=200, lambdas=[515e-9], zs=[2e-3], seed=711),
]


def run(ctx, P, n, T):
    field = ctx.rasterize(P, n).clone()
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    gfield = torch.empty_like(field)
    grads = ctx.backward(P, n, field, T, loss=loss, grad_field=gfield).clone()
    I, _ = ctx.propagate(field)
    torch.cuda.synchronize()
    return field, loss, gfield, grads, I


def test_static_context_matches_caller_workspace(O):
    for i, w in enumerate(CASES):
        H, W, C, n, L = w["H"], w["W"], w["C"], w["n"], len(w["zs"])
        say("static context", i, H, W, C, n)
        p = synth.params(w["seed"], n, H, W, C)
        T = torch.from_numpy(synth.target(w["seed"] + 1, C, H, W, L=L)).cuda()
        P = binding.pack(p, device="cuda")
        st = binding.Context(H, W, C, 8e-6, w["lambdas"], w["zs"], max_gaussians=n, static=True)
        assert st.workspace is None
        ref_ctx = binding.Context(H, W, C, 8e-6, w["lambdas"], w["zs"], max_gaussians=n)
        a = run(st, P, n, T)
        b = run(ref_ctx, P, n, T)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        assert st.read_status()[1]
        if i == 0:
            opt = O.Optics(H, W, C, 2 * H, 2 * W, 8e-6, w["lambdas"], w["zs"])
            ref = O.forward_backward(p, T.cpu().numpy(), opt)
            mask, _ = O.ambiguous_mask(p, opt, 1e-5)
            assert rel_l2(a[0].cpu().numpy(), ref["field"], mask) <= 1e-4
            assert abs(a[1][0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
            views = binding.unpack(a[3].cpu(), n, C)
            for k in binding.PARAM_KEYS:
                assert rel_l2(views[k].numpy(), ref["grads"][k]) <= 1e-3, k
            # one static context per device at a time
            with pytest.raises(binding.CghError) as e:
                binding.Context(H, W, C, 8e-6, w["lambdas"], w["zs"], max_gaussians=n,
                                static=True)
            assert e.value.status == 6
        st.close()
        ref_ctx.close()
    # too large for the static workspace: refused before any device work
    with pytest.raises(binding.CghError) as e:
        binding.Context(1080, 1920, 3, 8e-6, [639e-9, 515e-9, 473e-9], [5e-3],
                        max_gaussians=414720, static=True)
    assert e.value.status == 2
