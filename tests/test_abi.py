"""The C-ABI library loads and exports every entry point include/cgh.h declares;
host-only calls (configuration validation, workspace sizing) behave as the
header documents.  No device work is issued here."""
import ctypes
import os
import re

import pytest

from paper_2511_15022_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgh.h")


NET_HEADER = os.path.join(ROOT, "include", "cgh_net.h")
POH_HEADER = os.path.join(ROOT, "include", "cgh_poh.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgh_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(binding.EXPORTS)
    assert declared_functions(NET_HEADER) == sorted(binding.NET_EXPORTS)
    assert declared_functions(POH_HEADER) == sorted(binding.POH_EXPORTS)


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for name in (declared_functions() + declared_functions(NET_HEADER) +
                 declared_functions(POH_HEADER)):
        assert hasattr(L, name), name
    assert L.cgh_abi_version() == 4


def cfg(**kw):
    c = binding.cgh_config()
    c.height, c.width, c.channels = kw.get("H", 256), kw.get("W", 256), kw.get("C", 1)
    c.pad_height, c.pad_width = kw.get("Hp", 0), kw.get("Wp", 0)
    c.pitch_m = kw.get("pitch", 8e-6)
    for i, lam in enumerate(kw.get("lambdas", [515e-9] * min(c.channels, 4))):
        c.wavelength_m[i] = lam
    zs = kw.get("zs", [2e-3])
    c.num_planes = kw.get("L", len(zs))
    for i, z in enumerate(zs):
        c.z_m[i] = z
    c.support_sigma = kw.get("k", 3.0)
    c.max_gaussians = kw.get("n", 4096)
    c.max_pairs = kw.get("pairs", 0)
    c.flags = kw.get("flags", 0)
    c.aperture = kw.get("aperture", 0.0)
    c.tile_w, c.tile_h = kw.get("tile", (0, 0))
    c.batch = kw.get("B", 0)
    return c


def ws(c):
    size = ctypes.c_size_t(0)
    st = binding.lib().cgh_workspace_size(ctypes.byref(c), ctypes.byref(size))
    return st, size.value


def test_workspace_size_for_workloads():
    st, small = ws(cfg())
    assert st == 0 and small > 0
    st, big = ws(cfg(H=1080, W=1920, C=3, lambdas=[639e-9, 515e-9, 473e-9], zs=[5e-3],
                     n=414720))
    assert st == 0
    # the 1080p problem needs at least its [C][H][Wp] spectrum buffer and pair lists
    assert big > 3 * 1080 * 3840 * 8
    assert big < 2 * 1024 ** 3


def test_several_planes_accepted_and_sized():
    """Planes share the row spectrum; each further plane adds no per-plane
    spectrum copies beyond the two plane buffers (column output, adjoint sum)."""
    st1, one = ws(cfg(zs=[2e-3]))
    st3, three = ws(cfg(zs=[2e-3, 3e-3, -1e-3]))
    st8, eight = ws(cfg(zs=[1e-3 * (i + 1) for i in range(8)]))
    assert st1 == st3 == st8 == 0
    spec = 256 * 512 * 8  # [C][H][Wp] complex64 at C = 1
    assert three >= one + 2 * spec
    table = 257 * 257 * 8  # one quarter transfer table (Hp/2 + 1)(Wp/2 + 1) complex64
    # beyond three planes only the tables and the loss partials grow with L
    assert eight - three <= 5 * table + 8192


def test_full_loss_flag_reserves_the_ssim_buffers():
    """CGH_FULL_LOSS adds, per element of [L][C][H][W], the intensity (4 B) and
    the propagated field (8 B), three FP32 coefficient maps over the valid
    window positions, and the per-tile sums; nothing else changes."""
    kw = dict(H=200, W=120, C=3, lambdas=[639e-9, 515e-9, 473e-9], zs=[2e-3, 4e-3])
    st0, base = ws(cfg(**kw))
    st1, full = ws(cfg(flags=binding.CGH_FULL_LOSS, **kw))
    assert st0 == st1 == 0
    LC = 2 * 3
    need = LC * 200 * 120 * 12 + 3 * LC * 190 * 110 * 4
    assert need <= full - base <= need + 5 * 256 + 8 * LC * 2 * 7 * 4


def test_paper_alpha_flag_reserves_the_exponent_limits():
    """CGH_PAPER_ALPHA adds one (lo, hi) float pair per Gaussian slot (n + 1)."""
    st0, base = ws(cfg(n=5000))
    st1, pa = ws(cfg(n=5000, flags=binding.CGH_PAPER_ALPHA))
    assert st0 == st1 == 0
    assert 8 * 5001 <= pa - base <= 8 * 5001 + 256


@pytest.mark.parametrize("bad, status", [
    (dict(H=0), 1), (dict(W=9000), 1), (dict(C=5), 1), (dict(C=0), 1),
    (dict(Hp=514), 1),            # 514 = 2 * 257 does not factor into 2, 3, 5
    (dict(Hp=200), 1),            # smaller than H
    (dict(pitch=0.0), 1), (dict(lambdas=[-1.0]), 1), (dict(n=-1), 1),
    (dict(flags=8), 1), (dict(pairs=-5), 1),
    (dict(flags=1, H=10), 1), (dict(flags=1, W=10, Wp=20), 1),   # SSIM window is 11 x 11
    (dict(L=0), 1), (dict(zs=[1e-3] * 8, L=9), 1),   # 1 <= planes <= CGH_MAX_PLANES
    (dict(zs=[1e-3, float("nan")]), 1),
    (dict(aperture=-1.0), 1), (dict(aperture=float("inf")), 1),
    (dict(tile=(16, 0)), 1), (dict(tile=(0, 8)), 1),             # both or neither
    (dict(tile=(16, 32)), 5), (dict(tile=(64, 4)), 5), (dict(tile=(12, 12)), 5),
    (dict(B=65), 1), (dict(B=-1), 1),
    (dict(B=2, flags=1), 5),                                     # SSIM term: one hologram
])
def test_invalid_configs_are_rejected(bad, status):
    st, _ = ws(cfg(**bad))
    assert st == status
    assert binding.lib().cgh_last_error()


def test_check_finite_flag_reserves_nothing():
    st0, base = ws(cfg())
    st1, chk = ws(cfg(flags=binding.CGH_CHECK_FINITE))
    assert st0 == st1 == 0 and chk == base


def test_tile_shapes_and_batch_sizes():
    """Every supported tile shape is accepted; 8 x 8 tiles double the default
    pair capacity (16 n + 65536 pairs: keys and values twice, one partial
    record each).  A batch of B holograms multiplies the per-hologram
    buffers; only the twiddle tables are shared."""
    sizes = {}
    for t in binding.TILE_SHAPES:
        st, sizes[t] = ws(cfg(tile=t))
        assert st == 0, t
    assert sizes[(16, 16)] == ws(cfg())[1]
    # 8 x 8: 8 n more pairs (16 B of keys / values, 32 B of partials at C = 1),
    # about 4x the tile ranges
    extra = sizes[(8, 8)] - sizes[(16, 16)]
    assert 8 * 4096 * 48 <= extra <= 8 * 4096 * 48 + 4 * 1024 * 8 + 64 * 1024
    st1, one = ws(cfg(H=96, W=160, n=3000))
    st4, four = ws(cfg(H=96, W=160, n=3000, B=4))
    assert st1 == st4 == 0
    # shared: the 65536 spare pairs (keys, values, partials: 48 B each at
    # C = 1) and the twiddle tables; everything else is per hologram
    shared = 65536 * 48
    per = one - shared
    assert 2.9 * per < four - one < 3 * per + 64 * 1024


def test_null_arguments_are_rejected_without_device_work():
    L = binding.lib()
    assert L.cgh_workspace_size(None, None) == 1
    assert L.cgh_rasterize(None, None, 0, None, None) == 1
    assert L.cgh_backward(None, None, 0, None, None, None, None, None, None) == 1
    assert L.cgh_backward_full(None, None, 0, None, None, None, 0.005, None, None, None,
                               None) == 1
    assert L.cgh_step(None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None, 1, None) == 0
    assert L.cgh_step(None, None, None, None, 10, 1, 1e-3, 0.9, 0.999, 1e-8, None, 1, None) == 1
    c = cfg()
    out = ctypes.c_void_p()
    assert L.cgh_create(ctypes.byref(c), None, 0, None, ctypes.byref(out)) == 1
    lam = (ctypes.c_double * 1)(515e-9)
    assert L.cgh_set_optics(None, ctypes.cast(lam, ctypes.c_void_p),
                            ctypes.cast(lam, ctypes.c_void_p), None) == 1
    assert L.cgh_solve_create(None, None, 1, None, None, None, None, None, None, 10, 1e-3, 0.9,
                              0.999, 1e-8, None, ctypes.byref(out)) == 1
    assert L.cgh_solve_create(None, None, 1, None, None, None, None, None, None, 10, 1e-3, 0.9,
                              0.999, 1e-8, None, None) == 1
    assert L.cgh_solve_launch(None, None) == 1
    assert L.cgh_solve_destroy(None) == 0
    assert L.cgh_rasterize_lists(None, None, 0, None) == 1
    assert L.cgh_generation(None, None) == 1
    assert L.cgh_set_hologram_optics(None, 0, ctypes.cast(lam, ctypes.c_void_p),
                                     ctypes.cast(lam, ctypes.c_void_p), None) == 1


def test_net_argument_checks_and_workspace_sizes():
    """Host-side checks of the network entry points; no device work."""
    L = binding.lib()
    # 512 x 512, 32 -> 32: 16384 row chunks of 16 pixels in 512 splits; FP32
    # partials (512 x 9216) and bias partials (512 x 32), the channel-major
    # dL/dy (32 x 512 x 512 BF16) and the three shifted, padded input copies
    # (3 x 32 x 514 x 512 BF16), each part rounded up to 256 bytes
    ws = L.cgh_net_wgrad_workspace(512, 512, 32, 32)
    assert ws == 512 * 9216 * 4 + 512 * 32 * 4 + 32 * 512 * 512 * 2 + 3 * 32 * 514 * 512 * 2
    assert L.cgh_net_wgrad_workspace(0, 5, 8, 32) == 0
    # c1 not a multiple of 8, cout not a multiple of 8, missing outputs
    assert L.cgh_net_conv3x3(16, 6, 0, None, 0, 4, 4, 16, None, 32, 0, 16, None, None) == 1
    assert L.cgh_net_conv3x3(16, 8, 0, None, 0, 4, 4, 16, None, 12, 0, 16, None, None) == 1
    assert L.cgh_net_conv3x3(16, 8, 0, None, 0, 4, 4, 16, None, 32, 0, None, None, None) == 1
    # upsampled input with odd size; x2 given without channels
    assert L.cgh_net_conv3x3(16, 8, 1, None, 0, 5, 4, 16, None, 32, 0, 16, None, None) == 1
    assert L.cgh_net_conv3x3(16, 8, 0, 32, 0, 4, 4, 16, None, 32, 0, 16, None, None) == 1
    # workspace too small
    assert L.cgh_net_conv3x3_wgrad(16, 8, 0, None, 0, 64, 64, 16, 32, 16, None, 16, 8,
                                   None) == 2
    assert L.cgh_net_lattice_gather(16, 10, 10, 11, 3, 1, 16, None) == 1
    assert L.cgh_net_lattice_gather(16, 10, 10, 5, 3, 5, 16, None) == 1   # C > 4


def test_pack_unpack_layout_roundtrip():
    import numpy as np
    from paper_2511_15022_amd import synth
    p = synth.params(0, 10, 16, 16, 3)
    flat = binding.pack(p)
    assert flat.numel() == binding.param_count(10, 3)
    views = binding.unpack(flat, 10, 3)
    for k in binding.PARAM_KEYS:
        assert np.array_equal(views[k].numpy(), p[k])
