"""FP64 CPU oracle of the learned initialiser's network -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares nothing with the GPU package.

The network is a U-Net (Ronneberger, Fischer and Brox 2015) of 3x3
convolutions with zero padding, ReLU, 2x2 average pooling and nearest 2x
upsampling with skip concatenation, in NHWC layout with batch 1.  Its
precision contract is BF16 storage of weights and of the activations a
convolution reads, with sums in higher precision: ``bf16`` rounds to the
nearest BF16 value (ties to even), and the functions below take already
rounded inputs where the GPU does, so that the two differ only by the order
and precision of the sums.

Conventions (the GPU library uses the same ones):
  * conv weights w[co][ky][kx][ci]; out[y][x][co] = b[co] +
    sum_{ky,kx,ci} in[y + ky - 1][x + kx - 1][ci] w[co][ky][kx][ci]
    (in = 0 outside the image);
  * a convolution may read the concatenation [up(x1), x2] along channels,
    where up(x1) repeats each pixel of the half-resolution x1 over a 2x2
    block (x1 first);
  * pool: out[y][x] = mean of in[2y .. 2y + 1][2x .. 2x + 1].
"""
import numpy as np


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def up2(x):
    """Nearest 2x upsampling of [H][W][C]."""
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def up2_adjoint(g):
    """Adjoint of up2: sum of each 2x2 block."""
    H, W, C = g.shape
    return g.reshape(H // 2, 2, W // 2, 2, C).sum(axis=(1, 3))


def pool2(x):
    """2x2 average pooling of [H][W][C] (H, W even)."""
    H, W, C = x.shape
    return x.reshape(H // 2, 2, W // 2, 2, C).mean(axis=(1, 3))


def pool2_adjoint(g):
    return up2(g) / 4.0


def conv_input(x1, x2=None, up=False):
    """The tensor a convolution reads: [up(x1) or x1, x2] along channels."""
    a = up2(x1) if up else x1
    return a if x2 is None else np.concatenate([a, x2], axis=2)


def _shifted(x, ky, kx):
    """x[y + ky - 1][x + kx - 1] with zeros outside."""
    H, W, C = x.shape
    out = np.zeros_like(x)
    ys, yd = (slice(ky - 1, H), slice(0, H - ky + 1)) if ky >= 1 else (slice(0, H - 1), slice(1, H))
    xs, xd = (slice(kx - 1, W), slice(0, W - kx + 1)) if kx >= 1 else (slice(0, W - 1), slice(1, W))
    out[yd, xd] = x[ys, xs]
    return out


def conv3x3(x, w, b=None):
    """x [H][W][Ci], w [Co][3][3][Ci], b [Co] or None -> [H][W][Co]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:2] + (w.shape[0],))
    for ky in range(3):
        for kx in range(3):
            out += _shifted(x, ky, kx) @ w[:, ky, kx, :].T
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3x3_backward(x, w, gy):
    """Adjoints of conv3x3 at input x: returns (dL/dx, dL/dw, dL/db) for
    dL/dout = gy."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    gy = np.asarray(gy, np.float64)
    H, W, Ci = x.shape
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            xs = _shifted(x, ky, kx)
            gw[:, ky, kx, :] = gy.reshape(-1, gy.shape[2]).T @ xs.reshape(-1, Ci)
            # out[p] reads x[p + k - 1]: x[q] feeds out[q - k + 1]
            gx += _shifted(gy, 2 - ky, 2 - kx) @ w[:, ky, kx, :]
    return gx, gw, gy.sum(axis=(0, 1))


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------------------
# The U-Net: channel widths per level; every level has two convolutions, the
# decoder levels read [up(previous), skip].  ``arch`` lists the layers as
# (name, c_in_upsampled, c_in_skip, c_out, relu).
# ---------------------------------------------------------------------------
def architecture(c_in=8, widths=(32, 64, 128, 256), c_out=8):
    L = []
    prev = c_in
    for i, c in enumerate(widths):
        L.append((f"enc{i}a", prev, 0, c, True))
        L.append((f"enc{i}b", c, 0, c, True))
        prev = c
    for i in range(len(widths) - 2, -1, -1):
        c = widths[i]
        L.append((f"dec{i}a", prev, c, c, True))
        L.append((f"dec{i}b", c, 0, c, True))
        prev = c
    L.append(("head", prev, 0, c_out, False))
    return L


def init_weights(arch, seed):
    """He-normal weights (std sqrt(2 / (9 c_in))), zero biases, FP32."""
    rng = np.random.default_rng(seed)
    W = {}
    for name, cu, cs, co, _ in arch:
        ci = cu + cs
        W[name] = (rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))).astype(np.float32)
        W[name + ".b"] = np.zeros(co, np.float32)
    return W


def forward(arch, W, x, q=bf16):
    """x [H][W][c_in] (already BF16).  Returns (out [H][W][c_out], cache).
    Weights and every convolution input are BF16; the output of a
    convolution is kept in FP64 until it is stored as BF16 for the next one
    (after ReLU, and after pooling).  ``q``: the storage rounding (the
    identity gives the smooth FP64 network)."""
    bf16 = q
    nlev = sum(1 for n, *_ in arch if n.startswith("enc")) // 2
    cache = {"in": {}, "pre": {}}
    skips = []
    h = x
    k = 0
    for lev in range(nlev):
        for part in "ab":
            name, *_ = arch[k]
            cache["in"][name] = (h, None, False)
            z = conv3x3(h, bf16(W[name]), W[name + ".b"])
            cache["pre"][name] = z
            h = bf16(relu(z))
            k += 1
        if lev < nlev - 1:
            skips.append(h)
            h = bf16(pool2(h))
    for lev in range(nlev - 2, -1, -1):
        skip = skips[lev]
        name = arch[k][0]
        cache["in"][name] = (h, skip, True)
        z = conv3x3(conv_input(h, skip, up=True), bf16(W[name]), W[name + ".b"])
        cache["pre"][name] = z
        h = bf16(relu(z))
        k += 1
        name = arch[k][0]
        cache["in"][name] = (h, None, False)
        z = conv3x3(h, bf16(W[name]), W[name + ".b"])
        cache["pre"][name] = z
        h = bf16(relu(z))
        k += 1
    name = arch[k][0]
    cache["in"][name] = (h, None, False)
    out = conv3x3(h, bf16(W[name]), W[name + ".b"])
    return out, cache


def backward(arch, W, cache, g_out, q=bf16):
    """Gradients of every weight and bias for dL/dout = g_out.  The
    gradient a convolution's backward reads is rounded to BF16 first (the
    GPU feeds it to the same matrix units); ReLU passes it where the stored
    activation is positive."""
    bf16 = q
    grads = {}
    nlev = sum(1 for n, *_ in arch if n.startswith("enc")) // 2
    names = [a[0] for a in arch]

    def conv_back(name, g):
        h, skip, up = cache["in"][name]
        xin = conv_input(h, skip, up)
        gy = bf16(g)
        gx, gw, gb = conv3x3_backward(xin, bf16(W[name]), gy)
        grads[name], grads[name + ".b"] = gw, gb
        if skip is None:
            return gx, None
        cu = h.shape[2]
        return up2_adjoint(gx[:, :, :cu]), gx[:, :, cu:]

    def through_relu(name, g):
        return g * (cache["pre"][name] > 0)

    k = len(arch) - 1
    g, _ = conv_back(names[k], g_out)
    skip_g = [None] * (nlev - 1)
    for lev in range(0, nlev - 1):
        k -= 1
        g, _ = conv_back(names[k], through_relu(names[k], g))
        k -= 1
        g, gs = conv_back(names[k], through_relu(names[k], g))
        skip_g[lev] = gs
    for lev in range(nlev - 1, -1, -1):
        if lev < nlev - 1:
            g = pool2_adjoint(g) + skip_g[lev]
        for _ in range(2):
            k -= 1
            g, _ = conv_back(names[k], through_relu(names[k], g))
    return grads


# ---------------------------------------------------------------------------
# Gaussian lattice: Gaussian (i, j) of a G_y x G_x lattice sits at
# ((j + 1/2) W / G_x, (i + 1/2) H / G_y) and reads the network output (8 C
# channels, one block of 8 per colour channel) at the pixel containing that
# point.  Block 0 carries the shared geometry: 0, 1 offset of the mean
# (pixels), 2, 3 log-scale minus ln 2, 4 rotation, 7 opacity logit plus 1/2;
# block c carries colour c: 8 c + 5 amplitude minus 1/2, 8 c + 6 phase (so
# that zero outputs give the plain initialisation's scale, amplitude and
# opacity).
# ---------------------------------------------------------------------------
LOG_SCALE0, AMP0, OPACITY0 = np.log(2.0), 0.5, -0.5


def lattice(H, W, gy, gx):
    cy = (np.arange(gy) + 0.5) * H / gy
    cx = (np.arange(gx) + 0.5) * W / gx
    return np.meshgrid(cy, cx, indexing="ij")


def gather(out, H, W, gy, gx, C=1):
    """Network output [H][W][8 C] -> the library's parameter dict."""
    cy, cx = lattice(H, W, gy, gx)
    iy, ix = np.floor(cy).astype(int), np.floor(cx).astype(int)
    o = np.asarray(out, np.float64)[iy, ix].reshape(-1, 8 * C)
    mx = np.clip(cx.reshape(-1) + o[:, 0], 1e-3, W - 1e-3)
    my = np.clip(cy.reshape(-1) + o[:, 1], 1e-3, H - 1e-3)
    return {"mean_pre": np.stack([np.arctanh(2 * mx / W - 1), np.arctanh(2 * my / H - 1)], 1),
            "log_scale": o[:, 2:4] + LOG_SCALE0, "rotation": o[:, 4],
            "amplitude": o[:, 5::8] + AMP0, "phase": o[:, 6::8],
            "opacity_pre": o[:, 7] + OPACITY0}


def gather_adjoint(grads, out, H, W, gy, gx, C=1):
    """dL/d(network output) [H][W][8 C] from dL/d(parameters)."""
    cy, cx = lattice(H, W, gy, gx)
    iy, ix = np.floor(cy).astype(int).reshape(-1), np.floor(cx).astype(int).reshape(-1)
    o = np.asarray(out, np.float64)[iy, ix]
    mx = cx.reshape(-1) + o[:, 0]
    my = cy.reshape(-1) + o[:, 1]
    g = np.zeros((H, W, 8 * C))
    inx = (mx > 1e-3) & (mx < W - 1e-3)
    iny = (my > 1e-3) & (my < H - 1e-3)
    # d atanh(2m/W - 1)/dm = (2/W) / (1 - (2m/W - 1)^2)
    ux, uy = 2 * mx / W - 1, 2 * my / H - 1
    gm = np.asarray(grads["mean_pre"], np.float64)
    g[iy, ix, 0] = np.where(inx, gm[:, 0] * (2.0 / W) / (1 - ux * ux), 0.0)
    g[iy, ix, 1] = np.where(iny, gm[:, 1] * (2.0 / H) / (1 - uy * uy), 0.0)
    g[iy, ix, 2:4] = grads["log_scale"]
    g[iy, ix, 4] = grads["rotation"]
    g[iy, ix, 7] = grads["opacity_pre"]
    amp = np.asarray(grads["amplitude"]).reshape(-1, C)
    ph = np.asarray(grads["phase"]).reshape(-1, C)
    for c in range(C):
        g[iy, ix, 8 * c + 5] = amp[:, c]
        g[iy, ix, 8 * c + 6] = ph[:, c]
    return g
