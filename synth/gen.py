"""Generators for seeded uint8 search images and templates (numpy only).

Recipe (every draw comes from ``numpy.random.default_rng(seed)``):

* ``spectral_image``: white N(0,1) noise, shaped in the Fourier domain by
  f^(-beta/2) (so the power spectrum goes as 1/f^beta, DC removed), min-max
  rescaled to [0, 255] and rounded.
* ``add_rectangles``: one flat rectangle per 64x64 pixels of area, sides
  uniform in 4..40, grey level uniform in 170..255.
* ``add_lines``: one segment per 128x128 pixels of area, 3 px wide (pixels
  closer than 1.5 px to the segment), length uniform in [32, 512], dark
  (0..60) or bright (200..255) with equal probability.
* ``add_clouds``: a beta=4 spectral field c; alpha = clip((c - c90) /
  (c97 - c90), 0, 1) with c90/c97 its percentiles; pixel = round((1 -
  alpha) * I + alpha * 245).  About a tenth of the area is touched and the
  cores are flat and saturated.
* ``cut_template``: a block cut at a uniform valid location (re-drawn when
  its standard deviation is below 4), optionally given a contrast factor
  a in [0.8, 1.2] and brightness change b in [-0.2, 0.2] around its mean,
  plus N(0, sigma) noise, rounded and clipped to uint8.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 14073535


def config_seed(cfg: int, kind: str = "image", index: int = 0) -> int:
    """Seed of image ``index`` or template ``index`` of workload ``cfg`` (1-based)."""
    if kind == "image":
        return BASE_SEED + 1000 * cfg + index
    if kind == "template":
        return BASE_SEED + 1000 * cfg + 100 + index
    if kind == "arrivals":
        return BASE_SEED + 5999
    raise ValueError(kind)


def _spectral_field(rng: np.random.Generator, p: int, q: int, beta: float) -> np.ndarray:
    white = rng.standard_normal((p, q))
    spec = np.fft.rfft2(white)
    fy = np.fft.fftfreq(p)[:, None]
    fx = np.fft.rfftfreq(q)[None, :]
    f = np.hypot(fy, fx)
    f[0, 0] = 1.0
    shape = f ** (-beta / 2.0)
    shape[0, 0] = 0.0
    return np.fft.irfft2(spec * shape, s=(p, q))


def _to_u8(field: np.ndarray) -> np.ndarray:
    lo, hi = float(field.min()), float(field.max())
    if hi <= lo:
        return np.zeros(field.shape, np.uint8)
    return np.rint((field - lo) * (255.0 / (hi - lo))).astype(np.uint8)


def spectral_image(p: int, q: int, beta: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _to_u8(_spectral_field(rng, p, q, beta))


def add_rectangles(img: np.ndarray, rng: np.random.Generator, per_area: int = 64 * 64) -> np.ndarray:
    p, q = img.shape
    count = max(1, (p * q) // per_area)
    for _ in range(count):
        hh = int(rng.integers(4, 41))
        ww = int(rng.integers(4, 41))
        y0 = int(rng.integers(0, max(1, p - hh + 1)))
        x0 = int(rng.integers(0, max(1, q - ww + 1)))
        img[y0:y0 + hh, x0:x0 + ww] = np.uint8(rng.integers(170, 256))
    return img


def add_lines(img: np.ndarray, rng: np.random.Generator, per_area: int = 128 * 128) -> np.ndarray:
    p, q = img.shape
    count = max(1, (p * q) // per_area)
    for _ in range(count):
        length = float(rng.uniform(32.0, 512.0))
        ang = float(rng.uniform(0.0, np.pi))
        ya = float(rng.uniform(0, p - 1))
        xa = float(rng.uniform(0, q - 1))
        yb = ya + length * np.sin(ang)
        xb = xa + length * np.cos(ang)
        val = int(rng.integers(0, 61)) if rng.random() < 0.5 else int(rng.integers(200, 256))
        y_lo = max(0, int(np.floor(min(ya, yb) - 2)))
        y_hi = min(p, int(np.ceil(max(ya, yb) + 3)))
        x_lo = max(0, int(np.floor(min(xa, xb) - 2)))
        x_hi = min(q, int(np.ceil(max(xa, xb) + 3)))
        if y_lo >= y_hi or x_lo >= x_hi:
            continue
        yy, xx = np.mgrid[y_lo:y_hi, x_lo:x_hi].astype(np.float64)
        dy, dx = yb - ya, xb - xa
        t = ((yy - ya) * dy + (xx - xa) * dx) / (dy * dy + dx * dx)
        t = np.clip(t, 0.0, 1.0)
        dist = np.hypot(yy - (ya + t * dy), xx - (xa + t * dx))
        sub = img[y_lo:y_hi, x_lo:x_hi]
        sub[dist < 1.5] = np.uint8(val)
    return img


def add_clouds(img: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    p, q = img.shape
    c = _spectral_field(rng, p, q, 4.0)
    c90, c97 = np.percentile(c, [90.0, 97.0])
    alpha = np.clip((c - c90) / (c97 - c90), 0.0, 1.0)
    out = np.rint((1.0 - alpha) * img.astype(np.float64) + alpha * 245.0)
    return np.clip(out, 0, 255).astype(np.uint8)


def aerial_image(p: int, q: int, seed: int, beta=2.0, rectangles=True, lines=True,
                 clouds=False) -> np.ndarray:
    """Spectral texture plus optional rectangles, lines and clouds.

    ``beta`` may be a float or a (lo, hi) pair drawn uniformly per image.
    """
    rng = np.random.default_rng(seed)
    if isinstance(beta, (tuple, list)):
        beta = float(rng.uniform(beta[0], beta[1]))
    img = _to_u8(_spectral_field(rng, p, q, float(beta)))
    if rectangles:
        add_rectangles(img, rng)
    if lines:
        add_lines(img, rng)
    if clouds:
        img = add_clouds(img, rng)
    return np.ascontiguousarray(img)


def cut_template(img: np.ndarray, m: int, n: int, seed: int, noise_sigma: float,
                 affine: bool = False, min_std: float = 4.0):
    """Cut an m x n block at a seeded valid location; return (template, (y0, x0))."""
    rng = np.random.default_rng(seed)
    p, q = img.shape
    for _ in range(1000):
        y0 = int(rng.integers(0, p - m + 1))
        x0 = int(rng.integers(0, q - n + 1))
        blk = img[y0:y0 + m, x0:x0 + n].astype(np.float64)
        if blk.std() >= min_std:
            break
    if affine:
        a = float(rng.uniform(0.8, 1.2))
        b = float(rng.uniform(-0.2, 0.2))
        mu = blk.mean()
        blk = mu * (1.0 + b) + a * (blk - mu)
    if noise_sigma > 0:
        blk = blk + rng.normal(0.0, noise_sigma, blk.shape)
    tpl = np.clip(np.rint(blk), 0, 255).astype(np.uint8)
    return np.ascontiguousarray(tpl), (y0, x0)


def noise_template(m: int, n: int, seed: int) -> np.ndarray:
    """An independent beta=2 texture patch: a query with no true match."""
    return spectral_image(m, n, 2.0, seed)


def workload(cfg: int):
    """Inputs of the five named workloads.

    Returns a dict with ``images`` (list of uint8 arrays) and ``templates``
    (list of (template, (y0, x0) or None, image index)).
    """
    if cfg == 1:
        img = spectral_image(256, 256, 2.0, config_seed(1, "image", 0))
        t, loc = cut_template(img, 32, 32, config_seed(1, "template", 0), 5.0)
        return {"images": [img], "templates": [(t, loc, 0)]}
    if cfg == 2:
        img = aerial_image(2048, 2048, config_seed(2, "image", 0), beta=(1.8, 2.2))
        t, loc = cut_template(img, 64, 64, config_seed(2, "template", 0), 8.0)
        return {"images": [img], "templates": [(t, loc, 0)]}
    if cfg == 3:
        img = aerial_image(8192, 8192, config_seed(3, "image", 0), beta=2.0, clouds=True)
        sizes = [32, 64, 128, 32, 64, 128, 32, 64]
        tpls = []
        for k, s in enumerate(sizes):
            t, loc = cut_template(img, s, s, config_seed(3, "template", k), 10.0, affine=True)
            tpls.append((t, loc, 0))
        return {"images": [img], "templates": tpls}
    if cfg == 4:
        img = aerial_image(4096, 4096, config_seed(4, "image", 0), beta=2.0)
        rng = np.random.default_rng(config_seed(4, "template", 99))
        sizes = rng.choice([16, 32, 48, 64, 96, 128], size=64)
        tpls = []
        for k, s in enumerate(sizes):
            t, loc = cut_template(img, int(s), int(s), config_seed(4, "template", k), 6.0)
            tpls.append((t, loc, 0))
        return {"images": [img], "templates": tpls}
    if cfg == 5:
        imgs = [aerial_image(4096, 4096, config_seed(5, "image", 0), beta=2.0),
                aerial_image(4096, 4096, config_seed(5, "image", 1), beta=2.0),
                aerial_image(8192, 8192, config_seed(5, "image", 2), beta=2.0, clouds=True),
                aerial_image(8192, 8192, config_seed(5, "image", 3), beta=2.0, clouds=True)]
        return {"images": imgs, "templates": []}
    raise ValueError(f"unknown workload {cfg}")


def serving_queries(images, count: int, seed: int = None):
    """Query stream of the serving workload: square sizes uniform in 16..128,
    image chosen uniformly, half cut from the image + N(0, 8), half an
    independent beta=2 noise patch (no true match).  Returns a list of
    (template, image index, cut location or None)."""
    rng = np.random.default_rng(config_seed(5, "template", 0) if seed is None else seed)
    out = []
    for k in range(count):
        s = int(rng.integers(16, 129))
        j = int(rng.integers(0, len(images)))
        qseed = int(rng.integers(0, 2**31 - 1))
        if rng.random() < 0.5:
            t, loc = cut_template(images[j], s, s, qseed, 8.0)
            out.append((t, j, loc))
        else:
            out.append((noise_template(s, s, qseed), j, None))
    return out


def poisson_arrivals(count: int, qps: float, seed: int = None) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process at rate qps."""
    rng = np.random.default_rng(config_seed(5, "arrivals") if seed is None else seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
