"""The seeded generator is deterministic and draws what its recipe says."""

import numpy as np

from synth import aerial_image, config_seed, cut_template, spectral_image, workload


def test_same_seed_same_bytes():
    a = aerial_image(128, 160, 7, beta=(1.8, 2.2), clouds=True)
    b = aerial_image(128, 160, 7, beta=(1.8, 2.2), clouds=True)
    c = aerial_image(128, 160, 8, beta=(1.8, 2.2), clouds=True)
    assert a.dtype == np.uint8 and a.shape == (128, 160)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_spectral_image_uses_full_range_and_has_power_law_spectrum():
    img = spectral_image(256, 256, 2.0, 3).astype(np.float64)
    assert img.min() == 0 and img.max() == 255
    P = np.abs(np.fft.fft2(img - img.mean())) ** 2
    f = np.hypot(np.fft.fftfreq(256)[:, None], np.fft.fftfreq(256)[None, :])
    lo = P[(f > 0.02) & (f < 0.04)].mean()
    hi = P[(f > 0.16) & (f < 0.32)].mean()
    # 1/f^2 power: an 8x frequency ratio gives about 64x power
    assert 20 < lo / hi < 200


def test_template_cut_location_and_noise():
    img = spectral_image(200, 220, 2.0, 1)
    t, (y0, x0) = cut_template(img, 32, 24, 5, 0.0)
    assert np.array_equal(t, img[y0:y0 + 32, x0:x0 + 24])
    t2, loc2 = cut_template(img, 32, 24, 5, 5.0)
    assert loc2 == (y0, x0)
    d = t2.astype(int) - t.astype(int)
    assert 3.0 < d.std() < 7.0


def test_workload_one_shape():
    w = workload(1)
    img = w["images"][0]
    tpl, loc, idx = w["templates"][0]
    assert img.shape == (256, 256) and tpl.shape == (32, 32) and idx == 0
    assert config_seed(1) == 14073535 + 1000
