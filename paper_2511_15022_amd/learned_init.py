"""Learned initialiser: a U-Net that maps a target intensity to the parameters
of a lattice of Gaussians, the starting point of the optimisation of the
paper's Alg. 1 (the paper starts from random parameters, Sec. 4).

Host-side orchestration only: every arithmetic step runs in the library's
kernels (include/cgh_net.h for the network, include/cgh.h for the hologram
path, cgh_step for Adam); this module owns the device buffers (torch
tensors) and the order of the calls.

Network: 4 levels of two 3x3 convolutions with ReLU (widths 32, 64, 128,
256), 2x2 average pooling down, nearest upsampling with skip concatenation
up, and a 3x3 head to 8 output channels read by the Gaussian lattice.
Weights are kept in FP32 (Adam) with BF16 copies for the matrix cores.

Input features (8 channels, BF16): the target T, sqrt(T), and the real part,
imaginary part and modulus of sqrt(T) propagated back by -z with the
library's own band-limited angular-spectrum propagation, so that the network
sees the field a hologram has to produce at the SLM plane.
"""
import ctypes

import numpy as np
import torch

from . import binding

LOG2 = float(np.log(2.0))


def architecture(c_in=8, widths=(32, 64, 128, 256), c_out=8):
    """(name, c_in_upsampled, c_in_skip, c_out, relu) per convolution."""
    layers, prev = [], c_in
    for i, c in enumerate(widths):
        layers += [(f"enc{i}a", prev, 0, c, True), (f"enc{i}b", c, 0, c, True)]
        prev = c
    for i in range(len(widths) - 2, -1, -1):
        c = widths[i]
        layers += [(f"dec{i}a", prev, c, c, True), (f"dec{i}b", c, 0, c, True)]
        prev = c
    layers.append(("head", prev, 0, c_out, False))
    return layers


def he_weights(layers, seed):
    """He-normal weights (std sqrt(2 / (9 c_in))) and zero biases, FP32 numpy."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, cu, cs, co, _ in layers:
        ci = cu + cs
        out[name] = (rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))).astype(np.float32)
        out[name + ".b"] = np.zeros(co, np.float32)
    return out


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class UNet:
    """The network on one device for an H x W input (H, W divisible by 8)."""

    def __init__(self, H, W, widths=(32, 64, 128, 256), c_in=8, c_out=8, seed=0,
                 device="cuda"):
        if H % 8 or W % 8:
            raise ValueError("H and W must be multiples of 8 (three poolings)")
        self.H, self.W, self.dev = H, W, torch.device(device)
        self.widths = tuple(widths)
        self.layers = architecture(c_in, widths, c_out)
        self.L = binding.lib()
        # flat FP32 master weights: per layer [co][3][3][ci] then [co] bias
        self.off = {}
        n = 0
        for name, cu, cs, co, _ in self.layers:
            self.off[name] = (n, co * 9 * (cu + cs))
            n += co * 9 * (cu + cs)
            self.off[name + ".b"] = (n, co)
            n += co
        self.n_params = n
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.master = torch.zeros(n, **f32)
        self.grad = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.w16 = torch.zeros(n, dtype=torch.bfloat16, device=self.dev)
        self.wt16 = {name: torch.zeros(co * 9 * (cu + cs), dtype=torch.bfloat16, device=self.dev)
                     for name, cu, cs, co, _ in self.layers}
        self.t = 0
        # activations (BF16) per level l at (H >> l, W >> l)
        self.act = {}
        for name, cu, cs, co, _ in self.layers:
            lev = int(name[3]) if name != "head" else 0
            h, w = H >> lev, W >> lev
            if name != "head":
                self.act[name] = torch.zeros((h, w, co), dtype=torch.bfloat16, device=self.dev)
        self.pooled = {l: torch.zeros((H >> (l + 1), W >> (l + 1), widths[l]), dtype=torch.bfloat16,
                                      device=self.dev) for l in range(len(widths) - 1)}
        self.out = torch.zeros((H, W, c_out), **f32)
        ws = max(self.L.cgh_net_wgrad_workspace(H >> self._lev(nm), W >> self._lev(nm), cu + cs, co)
                 for nm, cu, cs, co, _ in self.layers)
        self.scratch = torch.empty(ws // 4 + 64, **f32)
        self.ws_bytes = ws
        self.set_weights(he_weights(self.layers, seed))

    @staticmethod
    def _lev(name):
        return 0 if name == "head" else int(name[3])

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def _chk(self, st):
        binding._check(st)

    def _view(self, t, name):
        o, n = self.off[name]
        return t[o:o + n]

    # -- weights ------------------------------------------------------------
    def set_weights(self, wd):
        """FP32 numpy weights by layer name (the layout above) -> device."""
        host = torch.zeros(self.n_params, dtype=torch.float32)
        for k, (o, n) in self.off.items():
            host[o:o + n] = torch.from_numpy(np.ascontiguousarray(wd[k], np.float32).reshape(-1))
        self.master.copy_(host.to(self.dev))
        self._refresh()

    def get_weights(self):
        host = self.master.cpu().numpy()
        out = {}
        for name, cu, cs, co, _ in self.layers:
            o, n = self.off[name]
            out[name] = host[o:o + n].reshape(co, 3, 3, cu + cs).copy()
            o, n = self.off[name + ".b"]
            out[name + ".b"] = host[o:o + n].copy()
        return out

    def _refresh(self):
        s = self._stream()
        self._chk(self.L.cgh_net_cast_bf16(_p(self.master), self.n_params, _p(self.w16), s))
        for name, cu, cs, co, _ in self.layers:
            if name == "enc0a":
                continue  # its input gradient is never needed
            self._chk(self.L.cgh_net_flip_weights(_p(self._view(self.w16, name)), co, cu + cs,
                                                  _p(self.wt16[name]), s))

    # -- passes ---------------------------------------------------------------
    def _conv(self, name, x1, up, x2, out32=None, out16=None):
        _, cu, cs, co, relu = next(l for l in self.layers if l[0] == name)
        lev = self._lev(name)
        h, w = self.H >> lev, self.W >> lev
        self._chk(self.L.cgh_net_conv3x3(_p(x1), cu, int(up), _p(x2), cs, h, w,
                                         _p(self._view(self.w16, name)),
                                         _p(self._view(self.master, name + ".b")), co, int(relu),
                                         _p(out32), _p(out16), self._stream()))

    def forward(self, x16):
        """x16: BF16 [H][W][c_in] -> FP32 [H][W][c_out] (self.out)."""
        nl = len(self.widths)
        h = x16
        for l in range(nl):
            self._conv(f"enc{l}a", h, False, None, out16=self.act[f"enc{l}a"])
            self._conv(f"enc{l}b", self.act[f"enc{l}a"], False, None, out16=self.act[f"enc{l}b"])
            h = self.act[f"enc{l}b"]
            if l < nl - 1:
                self._chk(self.L.cgh_net_pool2(_p(h), self.H >> l, self.W >> l, self.widths[l],
                                               _p(self.pooled[l]), self._stream()))
                h = self.pooled[l]
        for l in range(nl - 2, -1, -1):
            self._conv(f"dec{l}a", h, True, self.act[f"enc{l}b"], out16=self.act[f"dec{l}a"])
            self._conv(f"dec{l}b", self.act[f"dec{l}a"], False, None, out16=self.act[f"dec{l}b"])
            h = self.act[f"dec{l}b"]
        self._conv("head", h, False, None, out32=self.out)
        return self.out

    def backward(self, g_out, x16):
        """Weight gradients (self.grad) for dL/d(out) = g_out (FP32 [H][W][c_out])."""
        nl = len(self.widths)
        s = self._stream()
        dz = {}

        def zbuf(name):
            _, cu, cs, co, _ = next(l for l in self.layers if l[0] == name)
            lev = self._lev(name)
            return torch.empty(((self.H >> lev) * (self.W >> lev) * co,), dtype=torch.bfloat16,
                               device=self.dev)

        def wgrad(name, x1, up, x2, gy):
            _, cu, cs, co, _ = next(l for l in self.layers if l[0] == name)
            lev = self._lev(name)
            self._chk(self.L.cgh_net_conv3x3_wgrad(
                _p(x1), cu, int(up), _p(x2), cs, self.H >> lev, self.W >> lev, _p(gy), co,
                _p(self._view(self.grad, name)), _p(self._view(self.grad, name + ".b")),
                _p(self.scratch), self.ws_bytes, s))

        def dgrad(name, gy):
            _, cu, cs, co, _ = next(l for l in self.layers if l[0] == name)
            lev = self._lev(name)
            h, w = self.H >> lev, self.W >> lev
            gx = torch.empty((h, w, cu + cs), dtype=torch.float32, device=self.dev)
            self._chk(self.L.cgh_net_conv3x3(_p(gy), co, 0, None, 0, h, w, _p(self.wt16[name]),
                                             None, cu + cs, 0, _p(gx), None, s))
            return gx

        def relu_in(name, g, act):
            z = zbuf(name)
            self._chk(self.L.cgh_net_relu_grad(_p(g), _p(act), g.numel(), _p(z), s))
            return z

        # head (no ReLU on its output)
        z = relu_in("head", g_out, None)
        h_in = self.act["dec0b"] if nl > 1 else self.act["enc0b"]
        wgrad("head", h_in, False, None, z)
        g = dgrad("head", z)
        skip_g = {}
        for l in range(0, nl - 1):
            name = f"dec{l}b"
            z = relu_in(name, g, self.act[name])
            wgrad(name, self.act[f"dec{l}a"], False, None, z)
            g = dgrad(name, z)
            name = f"dec{l}a"
            z = relu_in(name, g, self.act[name])
            below = self.act[f"dec{l + 1}b"] if l + 1 < nl - 1 else self.act[f"enc{nl - 1}b"]
            wgrad(name, below, True, self.act[f"enc{l}b"], z)
            gx = dgrad(name, z)
            cu = self.widths[l + 1]
            h, w = self.H >> l, self.W >> l
            g = torch.empty((h // 2, w // 2, cu), dtype=torch.float32, device=self.dev)
            self._chk(self.L.cgh_net_up_adjoint(_p(gx), h, w, cu + self.widths[l], cu, _p(g), s))
            skip_g[l] = (gx, cu + self.widths[l], cu)
        for l in range(nl - 1, -1, -1):
            if l < nl - 1:
                gx, stride, off = skip_g[l]
                h, w = self.H >> l, self.W >> l
                g2 = torch.empty((h, w, self.widths[l]), dtype=torch.float32, device=self.dev)
                self._chk(self.L.cgh_net_grad_combine(_p(g), _p(gx), stride, off, h, w,
                                                      self.widths[l], _p(g2), s))
                g = g2
            name = f"enc{l}b"
            z = relu_in(name, g, self.act[name])
            wgrad(name, self.act[f"enc{l}a"], False, None, z)
            g = dgrad(name, z)
            name = f"enc{l}a"
            z = relu_in(name, g, self.act[name])
            x_in = x16 if l == 0 else self.pooled[l - 1]
            wgrad(name, x_in, False, None, z)
            if l > 0:
                g = dgrad(name, z)
        return self.grad

    def step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam on the FP32 master weights, then fresh BF16 and flipped copies."""
        self.t += 1
        binding.step(self.master, self.grad, self.m, self.v, self.t, lr, beta1, beta2, eps)
        self._refresh()


class Initializer:
    """Target intensity -> Gaussian parameters for one hologram geometry with
    C = len(wavelengths) colour channels sharing the Gaussians' geometry: a
    gy x gx lattice (one Gaussian per ``pixels_per_gaussian`` pixels), the
    U-Net (8 C input and output channels), and the contexts of the forward
    (z) and back (-z) propagations."""

    def __init__(self, H, W, pitch, wavelengths, z, pad=None, pixels_per_gaussian=5.0, seed=0,
                 device="cuda", widths=(32, 64, 128, 256), max_pairs=0):
        self.H, self.W, self.dev = H, W, torch.device(device)
        lams = list(wavelengths) if np.ndim(wavelengths) else [wavelengths]
        self.C = C = len(lams)
        g = np.sqrt(H * W / pixels_per_gaussian)
        self.gy = int(round(g * np.sqrt(H / W)))
        self.gx = int(round(H * W / pixels_per_gaussian / self.gy))
        self.n = self.gy * self.gx
        self.net = UNet(H, W, widths=widths, c_in=8 * C, c_out=8 * C, seed=seed, device=device)
        self.back = binding.Context(H, W, C, pitch, lams, [-z], pad=pad, max_gaussians=1,
                                    device=device)
        self.ctx = binding.Context(H, W, C, pitch, lams, [z], pad=pad, max_gaussians=self.n,
                                   max_pairs=max_pairs, device=device)
        self.x16 = torch.empty((H, W, 8 * C), dtype=torch.bfloat16, device=self.dev)
        self.field = torch.empty((C, H, W), dtype=torch.complex64, device=self.dev)
        self.params = torch.empty(self.n * (6 + 2 * C), dtype=torch.float32, device=self.dev)
        self.gparams = torch.empty_like(self.params)
        self.gnet = torch.empty((H, W, 8 * C), dtype=torch.float32, device=self.dev)
        self.loss = torch.zeros(2, dtype=torch.float64, device=self.dev)
        self.L = binding.lib()

    def _s(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def features(self, target):
        """target: FP32 [C][H][W] (device) -> the network input self.x16."""
        hw = self.H * self.W
        sq = torch.empty((self.C, self.H, self.W), dtype=torch.complex64, device=self.dev)
        binding._check(self.L.cgh_net_sqrt_field(_p(target), hw * self.C, _p(sq), self._s()))
        _, back = self.back.propagate(sq, intensity=False, field_out=True)
        binding._check(self.L.cgh_net_features(_p(target), _p(back), hw, self.C, _p(self.x16),
                                               self._s()))
        return self.x16

    def predict(self, target):
        """Gaussian parameters (library flat layout) for a target [C][H][W]."""
        self.net.forward(self.features(target))
        binding._check(self.L.cgh_net_lattice_gather(_p(self.net.out), self.H, self.W, self.gy,
                                                     self.gx, self.C, _p(self.params), self._s()))
        return self.params

    def grid(self):
        """The plain lattice ("grid") initialisation: zero network output."""
        zero = torch.zeros((self.H, self.W, 8 * self.C), dtype=torch.float32, device=self.dev)
        out = torch.empty_like(self.params)
        binding._check(self.L.cgh_net_lattice_gather(_p(zero), self.H, self.W, self.gy, self.gx,
                                                     self.C, _p(out), self._s()))
        return out

    def train_step(self, target, lr):
        """One step of end-to-end training: the network's parameters are
        rendered and propagated by the library, the MSE of the intensity
        against the target is backpropagated through the hologram path
        (cgh_backward), the lattice gather and the network, then Adam.
        Returns the device loss [L_MSE, PSNR] of this step's prediction."""
        params = self.predict(target)
        self.ctx.rasterize(params, self.n, self.field)
        self.ctx.backward(params, self.n, self.field, target.reshape(1, self.C, self.H, self.W),
                          loss=self.loss, grads=self.gparams)
        binding._check(self.L.cgh_net_lattice_scatter(_p(self.net.out), _p(self.gparams), self.H,
                                                      self.W, self.gy, self.gx, self.C,
                                                      _p(self.gnet), self._s()))
        self.net.backward(self.gnet, self.x16)
        self.net.step(lr)
        return self.loss


def scale_head(init, factor):
    """Multiply the head's weights (not its bias) by `factor`: with a small
    factor the untrained network's output is near zero, which is the plain
    lattice ("grid") initialisation."""
    wd = init.net.get_weights()
    wd["head"] = (wd["head"] * np.float32(factor)).astype(np.float32)
    init.net.set_weights(wd)


def train(init, targets, steps, lr, order_seed=0):
    """End-to-end training over a pool of device targets (FP32 [H][W] each),
    visited in a seeded random order.  Returns (per-step [L_MSE, PSNR] on the
    host, seconds)."""
    rng = np.random.default_rng(order_seed)
    order = rng.integers(0, len(targets), steps)
    log = torch.zeros((steps, 2), dtype=torch.float64, device=init.dev)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(init.dev)
    start.record()
    for i in range(steps):
        loss = init.train_step(targets[order[i]], lr)
        log[i].copy_(loss)
    stop.record()
    torch.cuda.synchronize(init.dev)
    return log.cpu().numpy(), start.elapsed_time(stop) / 1e3


def optimise(ctx, params, n, target, steps, lr=1e-3):
    """Adam (the plain optimiser) from `params` for `steps` steps on one
    target; returns (PSNR before each step, seconds at the end of each)."""
    P = params.clone()
    field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=P.device)
    G = torch.empty_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    log = torch.zeros((steps, 2), dtype=torch.float64, device=P.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    T = target.reshape(1, -1, *target.shape[-2:])
    torch.cuda.synchronize(P.device)
    ev[0].record()
    for i in range(steps):
        ctx.rasterize(P, n, field)
        ctx.backward(P, n, field, T, loss=log[i], grads=G)
        binding.step(P, G, M, V, i + 1, lr)
        ev[i + 1].record()
    torch.cuda.synchronize(P.device)
    t = np.array([ev[0].elapsed_time(ev[i + 1]) for i in range(steps)]) / 1e3
    return log[:, 1].cpu().numpy(), t
