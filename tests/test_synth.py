"""The seeded input generator: determinism, value ranges and the float32
hand-over shared by the oracle and the GPU path."""
import numpy as np

import synth


def test_deterministic_and_in_range():
    a = synth.clean_image(64, 48, 1)
    b = synth.clean_image(64, 48, 1)
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() <= 1.0
    assert not np.array_equal(a, synth.clean_image(64, 48, 2))


def test_noise_level():
    clean, noisy = synth.noisy_image(256, 256, 0.1, 3)
    assert abs(np.std(noisy - clean) - 0.1) < 0.005


def test_f32_handover_is_identical():
    f32, f64 = synth.noisy_f32(33, 17, 0.2, 4)
    assert f32.dtype == np.float32 and f64.dtype == np.float64
    assert np.array_equal(f32.astype(np.float64), f64)


def test_params_anchor_points():
    assert synth.params_for_sigma(0.1) == (0.15, 10.0)
    d, a = synth.params_for_sigma(0.07)
    assert 0.04 < d < 0.15 and 10.0 < a < 30.0
