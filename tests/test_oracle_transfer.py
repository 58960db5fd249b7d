"""Pins for the oracle's band-limited transfer function (Sec. 2 equation for H;
supplementary BLASM section): values fixed by the physics and by hand counts."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bandlimit_stress.txt")


def read_golden(path):
    vals = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = int(v)
    return vals


def test_dc_term_is_plane_wave_phase(O):
    lam, z = 515e-9, 2e-3
    H = O.transfer(512, 512, 8e-6, lam, z)
    # zero frequency: a plane wave along the axis picks up k z = 2 pi z / lambda
    expect = np.exp(1j * (2 * math.pi * z / lam % (2 * math.pi)))
    assert abs(H[0, 0] - expect) < 1e-9


def test_unit_modulus_in_band_and_conjugate_for_negative_distance(O):
    for (ny, nx) in [(512, 512), (36, 60)]:
        Hp = O.transfer(ny, nx, 8e-6, 639e-9, 5e-3)
        Hm = O.transfer(ny, nx, 8e-6, 639e-9, -5e-3)
        inband = np.abs(Hp) > 0
        assert np.all(np.abs(np.abs(Hp[inband]) - 1.0) < 1e-13)
        assert np.array_equal(inband, np.abs(Hm) > 0)
        assert np.max(np.abs(Hm - np.conj(Hp))) < 1e-9
        H0 = O.transfer(ny, nx, 8e-6, 639e-9, 0.0)
        assert np.allclose(H0, 1.0, atol=0)


def test_paraxial_limit_fixes_sign_and_frequency_scale(O):
    """For small f the phase relative to DC is -pi lambda z f^2 (Fresnel), with
    remainder below pi lambda^3 z f^4 / 4; this pins the frequency of each bin
    (natural order, bin k <-> k/(N dx)) and the sign of the exponent."""
    n, dx, lam, z = 512, 8e-6, 515e-9, 2e-3
    H = O.transfer(n, n, dx, lam, z)
    for (ky, kx) in [(0, 1), (0, 5), (3, 0), (7, 9), (0, n - 4), (n - 6, 2)]:
        sx = kx if kx < n // 2 else kx - n
        sy = ky if ky < n // 2 else ky - n
        f2 = (sx / (n * dx)) ** 2 + (sy / (n * dx)) ** 2
        rel = H[ky, kx] / H[0, 0]
        expect = -math.pi * lam * z * f2
        err = abs(np.angle(rel * np.exp(-1j * expect)))
        # remainder of sqrt(1 - x) = 1 - x/2 - x^2/8 (1 + O(x)), x = (lambda f)^2 <= 2e-3
        # plus FP64 rounding of the ~2.4e4 rad absolute phases of H[k] and H[0]
        assert err <= 1.01 * math.pi * lam ** 3 * z * f2 ** 2 / 4 + 3e-11


def test_natural_order_symmetry(O):
    H = O.transfer(48, 60, 8e-6, 473e-9, 7e-3)
    # H depends on f only through |f_x|, |f_y|: bin k and bin N-k coincide
    assert np.allclose(H[:, 1:], H[:, :0:-1], atol=0)
    assert np.allclose(H[1:, :], H[:0:-1, :], atol=0)


def test_band_limit_stress_count_matches_hand_count(O):
    g = read_golden(GOLDEN)
    H = O.transfer(512, 512, 8e-6, 515e-9, 300e-3)
    nz = np.abs(H) > 0
    assert int(nz.sum()) == g["nonzero_entries"]
    assert int(nz[0].sum()) == g["kept_bins_per_axis"]
    kept = np.flatnonzero(nz[0])
    signed = np.where(kept < 256, kept, kept - 512)
    assert signed.min() == -54 and signed.max() == 54


def test_band_limit_inactive_at_workload_geometries(O):
    # 1080p RGB geometry (padded 2160 x 3840, 8 um, 5 mm): every bin inside the band
    for lam in (639e-9, 515e-9, 473e-9):
        H = O.transfer(2160, 3840, 8e-6, lam, 5e-3)
        assert np.all(np.abs(H) > 0)
    H = O.transfer(512, 512, 8e-6, 515e-9, 2e-3)
    assert np.all(np.abs(H) > 0)


def test_aperture_keeps_the_lattice_points_inside_the_circle(O):
    """Alg. 3's circular aperture, centred on the zero frequency: radius 10 bins
    keeps the 305 lattice points with i^2 + j^2 < 100 (the 317 of the closed
    disk less the 12 on its rim: (+-10, 0), (0, +-10), (+-6, +-8), (+-8, +-6)),
    and inside it H is the unfiltered transfer function."""
    import numpy as np
    h0 = O.transfer(64, 64, 8e-6, 515e-9, 1e-3)
    h = O.transfer(64, 64, 8e-6, 515e-9, 1e-3, aperture=10.0)
    assert np.count_nonzero(h0) == 64 * 64           # the band limit does not bind here
    assert np.count_nonzero(h) == 305
    kept = h != 0
    assert np.array_equal(h[kept], h0[kept])
    assert h[0, 10] == 0 and h[0, 9] != 0 and h[6, 8] == 0 and h[63, 63] != 0
