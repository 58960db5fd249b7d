"""Phase-only hologram conversion of the complex Gaussian hologram (Sec. 3.3).

Host-side orchestration of the library's kernels (include/cgh_poh.h and
include/cgh.h); this module owns the device buffers and the call order.

* ``smooth``: the Smooth POH by double-phase coding of the rasterized field.
* ``RandomPOH``: the Random POH, a per-pixel phase optimised jointly with the
  Gaussians under L_extract; each step rasterizes the Gaussians, propagates
  their field and exp(j phi_rand) to every plane, forms the two adjoint seeds
  of L_extract, propagates them back, and takes an Adam step on the
  Gaussians (through the rasterizer adjoint) and one on the phase.
"""
import ctypes

import numpy as np
import torch

from . import binding

LAMBDA_COMP = 0.1
LAMBDA_FIELD = 0.01


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def smooth(field):
    """field: complex64 [C][H][W] -> (phases [C][H][W], exp(j phases))."""
    C, H, W = field.shape
    dev = field.device
    amax = torch.empty(C, dtype=torch.float32, device=dev)
    phase = torch.empty((C, H, W), dtype=torch.float32, device=dev)
    L = binding.lib()
    binding._check(L.cgh_poh_dpac(_p(field), C, H, W, _p(amax), _p(phase), _s(dev)))
    out = torch.empty((C, H, W), dtype=torch.complex64, device=dev)
    binding._check(L.cgh_poh_field(_p(phase), C * H * W, _p(out), _s(dev)))
    return phase, out


class RandomPOH:
    """Joint optimisation of the Gaussians (flat parameters, n of them, on
    context ``ctx``) and a random POH phase [C][H][W] under L_extract against
    ``target`` ([L][C][H][W]) with optional focal masks ([L][H][W])."""

    def __init__(self, ctx, params, n, target, mask=None, seed=0, lr=1e-3, lr_phase=0.1,
                 l_comp=LAMBDA_COMP, l_field=LAMBDA_FIELD):
        self.ctx, self.n = ctx, n
        self.dev = params.device
        C, H, W, L = ctx.C, ctx.H, ctx.W, ctx.L
        self.shape = (C, H, W)
        self.P = params.clone()
        rng = np.random.default_rng(seed)
        self.phase = torch.from_numpy(rng.uniform(0, 2 * np.pi, (C, H, W)).astype(np.float32)).to(self.dev)
        self.T = target.reshape(L, C, H, W)
        self.mask = mask
        self.lr, self.lr_phase, self.lc, self.lf = lr, lr_phase, l_comp, l_field
        z = lambda t: torch.zeros_like(t)
        self.G, self.M, self.V = z(self.P), z(self.P), z(self.P)
        self.gphase, self.Mp, self.Vp = z(self.phase), z(self.phase), z(self.phase)
        c64 = dict(dtype=torch.complex64, device=self.dev)
        self.field = torch.empty((C, H, W), **c64)
        self.hrand = torch.empty((C, H, W), **c64)
        self.gu = torch.empty((L, C, H, W), **c64)
        self.gur = torch.empty((L, C, H, W), **c64)
        self.gfield = torch.empty((C, H, W), **c64)
        self.ghrand = torch.empty((C, H, W), **c64)
        self.part = torch.empty(binding.lib().cgh_poh_extract_partials(L * C * H * W),
                                dtype=torch.float64, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.t = 0

    def gradients(self):
        """dL_extract/dparams (self.G) and dL_extract/dphase (self.gphase) at
        the current state; returns the propagated fields (u, u_rand)."""
        L = binding.lib()
        ctx, s = self.ctx, _s(self.dev)
        C, H, W = self.shape
        ctx.rasterize(self.P, self.n, self.field)
        _, u = ctx.propagate(self.field, intensity=False, field_out=True)
        binding._check(L.cgh_poh_field(_p(self.phase), C * H * W, _p(self.hrand), s))
        _, ur = ctx.propagate(self.hrand, intensity=False, field_out=True)
        binding._check(L.cgh_poh_extract_seed(
            _p(u), _p(ur), _p(self.T), _p(self.mask), ctx.L, C, H, W, self.lc, self.lf,
            _p(self.gu), _p(self.gur), _p(self.part), _p(self.loss), s))
        ctx.propagate_field_adjoint(self.gu, self.gfield)
        ctx.rasterize_adjoint(self.P, self.n, self.gfield, self.G)
        ctx.propagate_field_adjoint(self.gur, self.ghrand)
        binding._check(L.cgh_poh_phase_grad(_p(self.phase), _p(self.ghrand), C * H * W,
                                            _p(self.gphase), s))
        return u, ur

    def step(self):
        self.gradients()
        self.t += 1
        binding.step(self.P, self.G, self.M, self.V, self.t, self.lr)
        binding.step(self.phase, self.gphase, self.Mp, self.Vp, self.t, self.lr_phase)
        return self.loss
