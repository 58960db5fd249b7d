"""ctypes binding of libcgh (include/cgh.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and
the current stream.  If libcgh.so is missing, every call raises -- there is no
fallback path.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcgh.so")

MAX_CHANNELS = 4
MAX_PLANES = 8
CGH_FULL_LOSS = 1  # cgh_config.flags bit: workspace for cgh_backward_full
CGH_PAPER_ALPHA = 2  # cgh_config.flags bit: the Alg. 2 weight min(0.99, alpha G), skip < 1/255
CGH_CHECK_FINITE = 4  # cgh_config.flags bit: device check for NaN / Inf (cgh_read_status)
MAX_BATCH = 64
TILE_SHAPES = ((16, 16), (32, 8), (16, 8), (8, 8))  # rasterizer tiles (width, height)
PARAM_KEYS = ("mean_pre", "log_scale", "rotation", "amplitude", "phase", "opacity_pre")

KERNEL_CLASSES = {"preprocess": 1, "binning": 2, "raster": 3, "row_fft": 4, "col_pass": 5,
                  "row_loss": 6, "loss": 7, "raster_adjoint": 8, "preprocess_adjoint": 9}

STATUS = {0: "CGH_OK", 1: "CGH_ERR_INVALID_ARG", 2: "CGH_ERR_WORKSPACE", 3: "CGH_ERR_CAPACITY",
          4: "CGH_ERR_DEVICE", 5: "CGH_ERR_UNSUPPORTED", 6: "CGH_ERR_STATE",
          7: "CGH_ERR_NONFINITE"}


class CghError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class cgh_config(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("channels", ctypes.c_int32),
        ("pad_height", ctypes.c_int32), ("pad_width", ctypes.c_int32),
        ("pitch_m", ctypes.c_double),
        ("wavelength_m", ctypes.c_double * MAX_CHANNELS),
        ("num_planes", ctypes.c_int32),
        ("z_m", ctypes.c_double * MAX_PLANES),
        ("support_sigma", ctypes.c_float),
        ("max_gaussians", ctypes.c_int32),
        ("max_pairs", ctypes.c_int64),
        ("flags", ctypes.c_int32),
        ("aperture", ctypes.c_double),
        ("tile_w", ctypes.c_int32),
        ("tile_h", ctypes.c_int32),
        ("batch", ctypes.c_int32),
    ]


# (name, restype, argtypes) for every entry point of include/cgh.h
_VP = ctypes.c_void_p
_SIGS = [
    ("cgh_workspace_size", ctypes.c_int, [ctypes.POINTER(cgh_config), ctypes.POINTER(ctypes.c_size_t)]),
    ("cgh_create", ctypes.c_int, [ctypes.POINTER(cgh_config), _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("cgh_destroy", ctypes.c_int, [_VP]),
    ("cgh_create_static", ctypes.c_int, [ctypes.POINTER(cgh_config), _VP, ctypes.POINTER(_VP)]),
    ("cgh_rasterize", ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
    ("cgh_propagate", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("cgh_backward", ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cgh_backward_step", ctypes.c_int,
     [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32,
      ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]),
    ("cgh_backward_recon", ctypes.c_int,
     [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cgh_backward_full", ctypes.c_int,
     [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_float, _VP, _VP, _VP, _VP]),
    ("cgh_propagate_adjoint", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("cgh_propagate_field_adjoint", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("cgh_rasterize_adjoint", ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP]),
    ("cgh_rasterize_lists", ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP]),
    ("cgh_generation", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    ("cgh_step", ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP, ctypes.c_int32, _VP]),
    ("cgh_step_adan", ctypes.c_int,
     [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
      ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP,
      ctypes.c_int32, _VP]),
    ("cgh_get_transfer", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP]),
    ("cgh_read_status", ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_int64)]),
    ("cgh_profile_begin", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("cgh_profile_end", ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32)]),
    ("cgh_set_optics", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("cgh_set_hologram_optics", ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    ("cgh_solve_create", ctypes.c_int,
     [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_float,
      ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP, ctypes.POINTER(_VP)]),
    ("cgh_solve_launch", ctypes.c_int, [_VP, _VP]),
    ("cgh_solve_destroy", ctypes.c_int, [_VP]),
    ("cgh_last_error", ctypes.c_char_p, []),
    ("cgh_abi_version", ctypes.c_int32, []),
]
# entry points of include/cgh_net.h (the learned initialiser's network)
_I32, _I64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_NET_SIGS = [
    ("cgh_net_conv3x3", ctypes.c_int,
     [_VP, _I32, _I32, _VP, _I32, _I32, _I32, _VP, _VP, _I32, _I32, _VP, _VP, _VP]),
    ("cgh_net_flip_weights", ctypes.c_int, [_VP, _I32, _I32, _VP, _VP]),
    ("cgh_net_wgrad_workspace", ctypes.c_size_t, [_I32, _I32, _I32, _I32]),
    ("cgh_net_conv3x3_wgrad", ctypes.c_int,
     [_VP, _I32, _I32, _VP, _I32, _I32, _I32, _VP, _I32, _VP, _VP, _VP, _SZ, _VP]),
    ("cgh_net_cast_bf16", ctypes.c_int, [_VP, _I64, _VP, _VP]),
    ("cgh_net_relu_grad", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP]),
    ("cgh_net_pool2", ctypes.c_int, [_VP, _I32, _I32, _I32, _VP, _VP]),
    ("cgh_net_up_adjoint", ctypes.c_int, [_VP, _I32, _I32, _I32, _I32, _VP, _VP]),
    ("cgh_net_grad_combine", ctypes.c_int, [_VP, _VP, _I32, _I32, _I32, _I32, _I32, _VP, _VP]),
    ("cgh_net_lattice_gather", ctypes.c_int, [_VP, _I32, _I32, _I32, _I32, _I32, _VP, _VP]),
    ("cgh_net_lattice_scatter", ctypes.c_int,
     [_VP, _VP, _I32, _I32, _I32, _I32, _I32, _VP, _VP]),
    ("cgh_net_sqrt_field", ctypes.c_int, [_VP, _I64, _VP, _VP]),
    ("cgh_net_features", ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP]),
]
# entry points of include/cgh_poh.h (phase-only hologram conversion)
_POH_SIGS = [
    ("cgh_poh_dpac", ctypes.c_int, [_VP, _I32, _I32, _I32, _VP, _VP, _VP]),
    ("cgh_poh_field", ctypes.c_int, [_VP, _I64, _VP, _VP]),
    ("cgh_poh_phase_grad", ctypes.c_int, [_VP, _VP, _I64, _VP, _VP]),
    ("cgh_poh_extract_partials", ctypes.c_int64, [_I64]),
    ("cgh_poh_extract_seed", ctypes.c_int,
     [_VP, _VP, _VP, _VP, _I32, _I32, _I32, _I32, ctypes.c_float, ctypes.c_float, _VP, _VP, _VP,
      _VP, _VP]),
]
EXPORTS = tuple(name for name, _, _ in _SIGS)
POH_EXPORTS = tuple(name for name, _, _ in _POH_SIGS)
NET_EXPORTS = tuple(name for name, _, _ in _NET_SIGS)

_lib = None


def lib():
    """The loaded libcgh (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcgh.so not found at {LIB_PATH}; build it with "
                               "paper_2511_15022_amd/build.py (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS + _NET_SIGS + _POH_SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise CghError(status, lib().cgh_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t, dtype, numel, name, device):
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or t.device != device:
        raise ValueError(f"{name}: expected contiguous {dtype} with {numel} elements on {device}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def param_count(n, C):
    return n * (6 + 2 * C)


def pack(params, device=None):
    """Dict of the six pre-activation arrays -> one flat float32 tensor in the
    library's layout (mean_pre, log_scale, rotation, amplitude, phase, opacity_pre)."""
    parts = [torch.as_tensor(params[k], dtype=torch.float32).reshape(-1) for k in PARAM_KEYS]
    flat = torch.cat(parts)
    return flat.to(device) if device is not None else flat


def unpack(flat, n, C):
    """Views of a flat parameter (or gradient) tensor as the six arrays."""
    sizes = [2 * n, 2 * n, n, C * n, C * n, n]
    shapes = [(n, 2), (n, 2), (n,), (n, C), (n, C), (n,)]
    out, o = {}, 0
    for k, sz, sh in zip(PARAM_KEYS, sizes, shapes):
        out[k] = flat[o:o + sz].view(sh)
        o += sz
    return out


class Context:
    """One hologram problem, or a batch of ``batch`` holograms of one size, on
    one device (cgh_create / cgh_destroy).  The device workspace is a torch
    tensor owned by this object, or with ``static=True`` the library's static
    workspace (cgh_create_static: nothing is allocated; one such context per
    device at a time).  ``tile`` is the rasterizer tile (width, height), one
    of TILE_SHAPES (None: 16 x 16)."""

    def __init__(self, height, width, channels, pitch, wavelengths, zs, pad=None,
                 support_sigma=3.0, max_gaussians=0, max_pairs=0, full_loss=False,
                 paper_alpha=False, aperture=0.0, device="cuda", tile=None, batch=1,
                 check_finite=False, static=False):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.H, self.W, self.C = int(height), int(width), int(channels)
        zs = list(zs)
        wavelengths = list(wavelengths)
        if len(wavelengths) != self.C:
            raise ValueError("one wavelength per channel")
        cfg = cgh_config()
        cfg.height, cfg.width, cfg.channels = self.H, self.W, self.C
        hp, wp = pad if pad is not None else (0, 0)
        cfg.pad_height, cfg.pad_width = int(hp), int(wp)
        cfg.pitch_m = float(pitch)
        for i, lam in enumerate(wavelengths):
            cfg.wavelength_m[i] = float(lam)
        cfg.num_planes = len(zs)
        for i, z in enumerate(zs):
            cfg.z_m[i] = float(z)
        cfg.support_sigma = float(support_sigma)
        cfg.max_gaussians = int(max_gaussians)
        cfg.max_pairs = int(max_pairs)
        cfg.flags = ((CGH_FULL_LOSS if full_loss else 0) | (CGH_PAPER_ALPHA if paper_alpha else 0)
                     | (CGH_CHECK_FINITE if check_finite else 0))
        cfg.aperture = float(aperture)
        tw, th = tile if tile is not None else (0, 0)
        cfg.tile_w, cfg.tile_h = int(tw), int(th)
        cfg.batch = int(batch)
        self.B = int(batch)
        self.tile = (int(tw) or 16, int(th) or 16)
        self.cfg = cfg
        self.L = len(zs)
        self.Hp = cfg.pad_height or 2 * self.H
        self.Wp = cfg.pad_width or 2 * self.W
        size = ctypes.c_size_t(0)
        _check(lib().cgh_workspace_size(ctypes.byref(cfg), ctypes.byref(size)))
        self.workspace_bytes = size.value
        handle = ctypes.c_void_p()
        if static:
            # cgh_create_static: the library's static workspace, no allocation
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().cgh_create_static(ctypes.byref(cfg), _stream(self.device),
                                               ctypes.byref(handle)))
        else:
            self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                         device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            _check(lib().cgh_create(ctypes.byref(cfg), ctypes.c_void_p(aligned),
                                    self.workspace_bytes, _stream(self.device),
                                    ctypes.byref(handle)))
        self.handle = handle
        self.last_n = None

    def close(self):
        if getattr(self, "handle", None):
            lib().cgh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes -------------------------------------------------------------
    def field_shape(self):
        """[C][H][W], or [B][C][H][W] for a batch."""
        return (self.C, self.H, self.W) if self.B == 1 else (self.B, self.C, self.H, self.W)

    def plane_shape(self):
        """[L][C][H][W], or [L][B][C][H][W] for a batch."""
        if self.B == 1:
            return (self.L, self.C, self.H, self.W)
        return (self.L, self.B, self.C, self.H, self.W)

    def mask_shape(self):
        return (self.L, self.H, self.W) if self.B == 1 else (self.L, self.B, self.H, self.W)

    def param_count(self, n):
        """Floats of the parameter (or gradient) array of n Gaussians per hologram."""
        return self.B * param_count(n, self.C)

    def _field_numel(self):
        return self.B * self.C * self.H * self.W

    def _plane_numel(self):
        return self.L * self._field_numel()

    # -- entry points -------------------------------------------------------
    def rasterize(self, params, n, field=None):
        _need(params, torch.float32, self.param_count(n), "params", self.device)
        if field is None:
            field = torch.empty(self.field_shape(), dtype=torch.complex64, device=self.device)
        _need(field, torch.complex64, self._field_numel(), "field", self.device)
        _check(lib().cgh_rasterize(self.handle, _ptr(params), int(n), _ptr(field),
                                   _stream(self.device)))
        self.last_n = n
        return field

    def rasterize_lists(self, params, n):
        """cgh_rasterize_lists: rebuild the tile lists of ``params`` (no field)."""
        _need(params, torch.float32, self.param_count(n), "params", self.device)
        _check(lib().cgh_rasterize_lists(self.handle, _ptr(params), int(n), _stream(self.device)))
        self.last_n = n

    def generation(self):
        """cgh_generation: rasterize / rasterize_lists calls made so far."""
        g = ctypes.c_int64(0)
        _check(lib().cgh_generation(self.handle, ctypes.byref(g)))
        return g.value

    def propagate(self, field, intensity=True, field_out=False):
        _need(field, torch.complex64, self._field_numel(), "field", self.device)
        I = torch.empty(self.plane_shape(), dtype=torch.float32, device=self.device) if intensity else None
        u = torch.empty(self.plane_shape(), dtype=torch.complex64, device=self.device) if field_out else None
        _check(lib().cgh_propagate(self.handle, _ptr(field), _ptr(I), _ptr(u), _stream(self.device)))
        return I, u

    def backward(self, params, n, field, target, loss=None, grad_field=None, grads=None,
                 mask=None, ssim_weight=None):
        """L_MSE backward; with ``mask`` ([L][H][W]) the L_recon backward; with
        ``ssim_weight`` (a context made with ``full_loss=True``) the final loss
        L_recon (or L_MSE) + ssim_weight L_SSIM."""
        _need(params, torch.float32, self.param_count(n), "params", self.device)
        _need(field, torch.complex64, self._field_numel(), "field", self.device)
        _need(target, torch.float32, self._plane_numel(), "target", self.device)
        if grads is None:
            grads = torch.empty_like(params)
        if loss is not None:
            _need(loss, torch.float64, 2 * self.B, "loss", self.device)
        if grad_field is not None:
            _need(grad_field, torch.complex64, self._field_numel(), "grad_field", self.device)
        if mask is not None:
            _need(mask, torch.float32, self.L * self.B * self.H * self.W, "mask", self.device)
        if ssim_weight is not None:
            _check(lib().cgh_backward_full(self.handle, _ptr(params), int(n), _ptr(field),
                                           _ptr(target), _ptr(mask), float(ssim_weight),
                                           _ptr(loss), _ptr(grad_field), _ptr(grads),
                                           _stream(self.device)))
        elif mask is None:
            _check(lib().cgh_backward(self.handle, _ptr(params), int(n), _ptr(field),
                                      _ptr(target), _ptr(loss), _ptr(grad_field), _ptr(grads),
                                      _stream(self.device)))
        else:
            _check(lib().cgh_backward_recon(self.handle, _ptr(params), int(n), _ptr(field),
                                            _ptr(target), _ptr(mask), _ptr(loss),
                                            _ptr(grad_field), _ptr(grads),
                                            _stream(self.device)))
        return grads

    def backward_step(self, params, n, field, target, m, v, t, lr, beta1=0.9, beta2=0.999,
                      eps=1e-8, loss=None, grad_field=None, grads=None):
        """cgh_backward_step: the L_MSE backward and the Adam update of ``params``
        (in place, with moments ``m``, ``v``) in one pass of the per-Gaussian
        adjoint stage.  ``grads`` (optional) receives dL/dparams."""
        _need(params, torch.float32, self.param_count(n), "params", self.device)
        _need(m, torch.float32, self.param_count(n), "m", self.device)
        _need(v, torch.float32, self.param_count(n), "v", self.device)
        _need(field, torch.complex64, self._field_numel(), "field", self.device)
        _need(target, torch.float32, self._plane_numel(), "target", self.device)
        if grads is not None:
            _need(grads, torch.float32, self.param_count(n), "grads", self.device)
        if loss is not None:
            _need(loss, torch.float64, 2 * self.B, "loss", self.device)
        if grad_field is not None:
            _need(grad_field, torch.complex64, self._field_numel(), "grad_field", self.device)
        _check(lib().cgh_backward_step(self.handle, _ptr(params), int(n), _ptr(field),
                                       _ptr(target), _ptr(loss), _ptr(grad_field), _ptr(grads),
                                       _ptr(m), _ptr(v), int(t), float(lr), float(beta1),
                                       float(beta2), float(eps), _stream(self.device)))

    def propagate_field_adjoint(self, grad_u, grad_field=None):
        """cgh_propagate_field_adjoint: sum over planes of P^H grad_u."""
        _need(grad_u, torch.complex64, self._plane_numel(), "grad_u", self.device)
        if grad_field is None:
            grad_field = torch.empty(self.field_shape(), dtype=torch.complex64, device=self.device)
        _need(grad_field, torch.complex64, self._field_numel(), "grad_field", self.device)
        _check(lib().cgh_propagate_field_adjoint(self.handle, _ptr(grad_u), _ptr(grad_field),
                                                 _stream(self.device)))
        return grad_field

    def propagate_adjoint(self, field, grad_intensity, grad_field=None):
        _need(field, torch.complex64, self._field_numel(), "field", self.device)
        _need(grad_intensity, torch.float32, self._plane_numel(), "grad_intensity", self.device)
        if grad_field is None:
            grad_field = torch.empty(self.field_shape(), dtype=torch.complex64, device=self.device)
        _check(lib().cgh_propagate_adjoint(self.handle, _ptr(field), _ptr(grad_intensity),
                                           _ptr(grad_field), _stream(self.device)))
        return grad_field

    def rasterize_adjoint(self, params, n, grad_field, grads=None):
        _need(params, torch.float32, self.param_count(n), "params", self.device)
        _need(grad_field, torch.complex64, self._field_numel(), "grad_field", self.device)
        if grads is None:
            grads = torch.empty_like(params)
        _check(lib().cgh_rasterize_adjoint(self.handle, _ptr(params), int(n), _ptr(grad_field),
                                           _ptr(grads), _stream(self.device)))
        return grads

    def set_hologram_optics(self, hologram, wavelengths, zs, stream=None):
        """cgh_set_hologram_optics: new optics for one hologram of a batch."""
        if len(wavelengths) != self.C or len(zs) != self.L:
            raise ValueError(f"need {self.C} wavelengths and {self.L} distances")
        lam = (ctypes.c_double * self.C)(*[float(x) for x in wavelengths])
        zz = (ctypes.c_double * self.L)(*[float(x) for x in zs])
        st = _stream(self.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().cgh_set_hologram_optics(self.handle, int(hologram),
                                             ctypes.cast(lam, ctypes.c_void_p),
                                             ctypes.cast(zz, ctypes.c_void_p), st))

    def get_transfer(self, channel=0, plane=0):
        out = torch.empty((self.Hp // 2 + 1, self.Wp // 2 + 1), dtype=torch.complex64,
                          device=self.device)
        _check(lib().cgh_get_transfer(self.handle, int(channel), int(plane), _ptr(out),
                                      _stream(self.device)))
        return out

    def set_optics(self, wavelengths, zs, stream=None):
        """cgh_set_optics: new wavelengths ([C]) and distances ([L]) for this
        context; the transfer tables are rebuilt on ``stream`` (default: the
        current stream)."""
        if len(wavelengths) != self.C or len(zs) != self.L:
            raise ValueError(f"need {self.C} wavelengths and {self.L} distances")
        lam = (ctypes.c_double * self.C)(*[float(x) for x in wavelengths])
        zz = (ctypes.c_double * self.L)(*[float(x) for x in zs])
        st = _stream(self.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().cgh_set_optics(self.handle, ctypes.cast(lam, ctypes.c_void_p),
                                    ctypes.cast(zz, ctypes.c_void_p), st))

    def profile_begin(self, kernel_class):
        _check(lib().cgh_profile_begin(self.handle, int(KERNEL_CLASSES[kernel_class])))

    def profile_end(self):
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int32(0)
        _check(lib().cgh_profile_end(self.handle, _stream(self.device), ctypes.byref(ms),
                                     ctypes.byref(cnt)))
        return ms.value, cnt.value

    def read_status(self, raise_on_overflow=True):
        pairs = ctypes.c_int64(0)
        st = lib().cgh_read_status(self.handle, _stream(self.device), ctypes.byref(pairs))
        if st != 0 and (raise_on_overflow or st != 3):
            _check(st)
        return pairs.value, st == 0


class Solve:
    """cgh_solve_*: ``steps`` Adam steps of L_MSE on ``ctx`` captured once as a
    HIP graph over the given buffers (params and target are read when a launch
    starts; params holds the result).  The solve owns its field, gradient,
    moment and loss-log buffers (``self.loss_log``: [steps][2] doubles, or
    [steps][B][2] for a batch)."""

    def __init__(self, ctx, params, n, target, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
        dev = ctx.device
        _need(params, torch.float32, ctx.param_count(n), "params", dev)
        _need(target, torch.float32, ctx._plane_numel(), "target", dev)
        self.ctx, self.n, self.steps = ctx, n, steps
        self.params, self.target = params, target
        self.field = torch.empty(ctx.field_shape(), dtype=torch.complex64, device=dev)
        self.grads = torch.empty_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        shape = (steps, 2) if ctx.B == 1 else (steps, ctx.B, 2)
        self.loss_log = torch.zeros(shape, dtype=torch.float64, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        handle = ctypes.c_void_p()
        _check(lib().cgh_solve_create(ctx.handle, _ptr(params), int(n), _ptr(target),
                                      _ptr(self.field), _ptr(self.grads), _ptr(self.m),
                                      _ptr(self.v), _ptr(self.loss_log), int(steps), float(lr),
                                      float(beta1), float(beta2), float(eps),
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(handle)))
        self.handle = handle
        ctx.last_n = n

    def launch(self, stream=None):
        """Enqueues one solve on ``stream`` (default: the stream it was made on)."""
        s = self.stream if stream is None else stream
        _check(lib().cgh_solve_launch(self.handle, ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().cgh_solve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, lr_groups=None,
         channels=1):
    """cgh_step: in-place Adam over flat tensors of equal size."""
    for name, x in (("grads", grads), ("m", m), ("v", v)):
        _need(x, torch.float32, params.numel(), name, params.device)
    _need(params, torch.float32, params.numel(), "params", params.device)
    groups = None
    if lr_groups is not None:
        groups = (ctypes.c_float * 6)(*[float(x) for x in lr_groups])
    _check(lib().cgh_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), int(t),
                          float(lr), float(beta1), float(beta2), float(eps),
                          ctypes.cast(groups, ctypes.c_void_p) if groups is not None else None,
                          int(channels), _stream(params.device)))


def step_adan(params, grads, m, d, s, prev_grads, t, lr, beta1=0.98, beta2=0.92, beta3=0.99,
              eps=1e-8, weight_decay=0.0, lr_groups=None, channels=1):
    """cgh_step_adan: in-place Adan over flat tensors of equal size."""
    for name, x in (("grads", grads), ("m", m), ("d", d), ("s", s), ("prev_grads", prev_grads)):
        _need(x, torch.float32, params.numel(), name, params.device)
    _need(params, torch.float32, params.numel(), "params", params.device)
    groups = None
    if lr_groups is not None:
        groups = (ctypes.c_float * 6)(*[float(x) for x in lr_groups])
    _check(lib().cgh_step_adan(_ptr(params), _ptr(grads), _ptr(m), _ptr(d), _ptr(s),
                               _ptr(prev_grads), params.numel(), int(t), float(lr), float(beta1),
                               float(beta2), float(beta3), float(eps), float(weight_decay),
                               ctypes.cast(groups, ctypes.c_void_p) if groups is not None else None,
                               int(channels), _stream(params.device)))
