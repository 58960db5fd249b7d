"""The seeded generators are deterministic, shaped and ranged as documented."""
import math

import numpy as np

from paper_2511_15022_amd import synth


def test_params_deterministic_and_ranged():
    a = synth.params(0, 1000, 64, 96, 3)
    b = synth.params(0, 1000, 64, 96, 3)
    for k in synth.PARAM_KEYS:
        assert a[k].dtype == np.float32 and a[k].flags.c_contiguous
        assert np.array_equal(a[k], b[k])
    assert a["mean_pre"].shape == (1000, 2) and a["amplitude"].shape == (1000, 3)
    mu_x = (np.tanh(a["mean_pre"][:, 0].astype(np.float64)) + 1) / 2 * 96
    assert mu_x.min() >= 0 and mu_x.max() < 96
    assert abs(np.mean(a["log_scale"]) - math.log(2)) < 0.03
    assert a["rotation"].min() >= 0 and a["rotation"].max() < math.pi
    assert np.all(a["opacity_pre"] == np.float32(-0.5))
    c = synth.params(1, 1000, 64, 96, 3)
    assert not np.array_equal(a["phase"], c["phase"])


def test_target_deterministic_and_ranged():
    t = synth.target(1, 2, 50, 70, L=2)
    assert t.shape == (2, 2, 50, 70) and t.dtype == np.float32
    assert t.min() >= 0 and t.max() <= 1 and t.std() > 0.05
    assert np.array_equal(t, synth.target(1, 2, 50, 70, L=2))
