"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Integer sums, locations, counts, group sizes, traces and blurred images must
be bit-exact; the binary64 rho of the answer is bit-identical (same
correctly-rounded operations on the same exact integers); binary32 rho is
within 1e-6 of the oracle's binary64 value.
"""

import math

import numpy as np
import pytest

import oracle as O
from synth import aerial_image, cut_template, spectral_image, workload

pytestmark = pytest.mark.gpu

Z = pytest.importorskip("paper_1407_3535_amd")

RHO32_TOL = 1e-6
KEYS = ("y", "x", "rho", "num", "den_t", "den_r")


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = Z.Searcher(0)
    yield s
    s.close()


def same_answer(g, o, what=""):
    for k in KEYS:
        assert g[k] == o[k], f"{what}: {k} gpu={g[k]} oracle={o[k]}"
    assert abs(g["rho32"] - o["rho"]) <= RHO32_TOL, what


def same_counts(g, o, what=""):
    for k in ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed", "group_h", "group_w"):
        assert g[k] == o[k], f"{what}: {k} gpu={g[k]} oracle={o[k]}"
    assert g["best0"] == o["best0"], what


def small_cases():
    out = []
    rng = np.random.default_rng(7)
    shapes = [(40, 50, 7, 9), (64, 64, 16, 16), (33, 70, 5, 13), (90, 47, 12, 10), (300, 280, 32, 32),
              (130, 129, 21, 3), (50, 50, 50, 50), (17, 300, 4, 65)]
    for k, (p, q, m, n) in enumerate(shapes):
        img = spectral_image(p, q, 2.0, 1000 + k)
        if k % 3 == 1:
            img[: p // 3, : q // 3] = 211  # flat block: degenerate windows
        y0, x0 = int(rng.integers(0, p - m + 1)), int(rng.integers(0, q - n + 1))
        tpl = np.clip(img[y0:y0 + m, x0:x0 + n].astype(int) + rng.integers(-5, 6, (m, n)), 0, 255).astype(np.uint8)
        if tpl.std() == 0:
            tpl[0, 0] ^= 1
        out.append((img, tpl))
    return out


CASES = small_cases()


@pytest.mark.parametrize("k", range(len(CASES)))
def test_full_maps_bit_exact(S, k):
    img, tpl = CASES[k]
    print(f"case {k} img {img.shape} tpl {tpl.shape}", flush=True)
    i = S.load(img)
    num, dr, rho32 = Z.zts_debug_full_map(S.ctx, i, img.shape, tpl)
    o = O.full_search(img, tpl, maps=True)
    assert np.array_equal(num, o["num_map"])
    assert np.array_equal(dr, o["dr_map"])
    assert np.abs(rho32.astype(np.float64) - o["rho_map"]).max() <= RHO32_TOL
    g = S.search(i, tpl, "full")
    same_answer(g, o, f"full case {k}")
    assert g["n_computed"] == g["n_locations"] == o["rho_map"].size
    same_answer(S.search(i, tpl, "full_mfma"), o, f"full_mfma case {k}")
    S.unload(i)


def test_full_mfma_four_row_groups(S):
    """A 2048x4096 image with one 64x64 template: the single-template MFMA kernel runs 64-row blocks
    here (128-row blocks from 4096x4096 up, 32-row blocks on the small cases).  The answer equals the
    v_dot4 exhaustive search's, and the oracle recomputes the exact sums at it."""
    img = spectral_image(2048, 4096, 2.0, 4096)
    tpl, _ = cut_template(img, 64, 64, 4097, 6.0)
    i = S.load(img)
    g = S.search(i, tpl, "full_mfma")
    f = S.search(i, tpl, "full")
    for k in KEYS:
        assert g[k] == f[k], k
    y, x = g["y"], g["x"]
    sub = O.full_search(img[y:y + 64, x:x + 64], tpl)
    assert (g["num"], g["den_t"], g["den_r"], g["rho"]) == (sub["num"], sub["den_t"], sub["den_r"], sub["rho"])
    S.unload(i)


def test_workload1_full_and_te(S):
    w = workload(1)
    img = w["images"][0]
    tpl, loc, _ = w["templates"][0]
    i = S.load(img)
    o = O.full_search(img, tpl)
    same_answer(S.search(i, tpl, "full"), o, "full")
    assert (o["y"], o["x"]) == loc
    ot = O.te_search(img, tpl, 3, 3, decision=True)
    g, dec = S.search(i, tpl, "te_fixed", decision=True, group_h=3, group_w=3)
    same_answer(g, o, "te 3x3")
    same_counts(g, ot, "te 3x3")
    assert np.array_equal(dec, ot["decision"])
    S.unload(i)


@pytest.mark.parametrize("k", range(len(CASES)))
@pytest.mark.parametrize("hw", [(3, 3), (4, 2), (5, 5)])
def test_autocorr_bit_exact(S, k, hw):
    img, tpl = CASES[k]
    m, n = tpl.shape
    h, w = hw
    i = S.load(img)
    g = Z.zts_debug_autocorr(S.ctx, i, img.shape, m, n, h, w)
    o = O.autocorr(img, m, n, h, w)
    for a, b in zip(g, o):
        assert np.array_equal(a, b)
    S.unload(i)


@pytest.mark.parametrize("taps", ["paper", 0.5, 0.5 * math.sqrt(3), 1.5, 0.5 * math.sqrt(11)])
def test_blur_bit_exact(S, taps):
    img = aerial_image(97, 131, 5)
    t = O.PAPER_W if taps == "paper" else O.gauss_taps(taps)[0]
    assert np.array_equal(Z.zts_debug_blur(S.ctx, img, t), O.blur(img, t))


@pytest.mark.parametrize("k", range(len(CASES)))
@pytest.mark.parametrize("hw,radius", [((3, 3), 0), ((4, 6), 0), ((5, 5), 2), ((1, 1), 0), ((2, 3), 1), ((12, 14), 1)])
def test_te_fixed_parity(S, k, hw, radius):
    img, tpl = CASES[k]
    h, w = hw
    print(f"case {k} {img.shape} {tpl.shape} hw={hw} r={radius}", flush=True)
    i = S.load(img)
    full = O.full_search(img, tpl)
    ot = O.te_search(img, tpl, h, w, decision=True, radius=radius)
    g, dec = S.search(i, tpl, "te_fixed", decision=True, group_h=h, group_w=w, refine_radius=radius)
    same_answer(g, full, "te vs full")
    same_counts(g, ot, "te vs oracle te")
    assert np.array_equal(dec, ot["decision"])
    S.unload(i)


# Alg. 2 as printed, then Prop. 3.1's two-root estimate at assumed template-to-centre correlations and the
# ascent over non-square group sizes.
EGS_CASES = [(0, {}), (1, {}), (2, {}), (0, dict(egs_estimate=1)), (1, dict(egs_estimate=1, rho_tc=0.3)),
             (2, dict(egs_shape=1)), (0, dict(egs_estimate=1, rho_tc=-0.25, egs_shape=1))]


@pytest.mark.parametrize("case", EGS_CASES, ids=[f"egs{k}" for k in range(len(EGS_CASES))])
def test_egs_parity(S, case):
    seed, kw = case
    img = aerial_image(160, 200, 300 + seed, beta=(1.8, 2.6))
    m = n = 16
    i = S.load(img)
    info = S.prepare(i, m, n, "egs", **kw)
    oe = O.egs(img, m, n, estimate=kw.get("egs_estimate", 0), rho_tc=kw.get("rho_tc", 0.0),
               shape=kw.get("egs_shape", 0))
    assert (info["h"], info["w"], info["cost"]) == (oe["h"], oe["w"], oe["cost"])
    assert info["egs"] == oe["trace"]
    for k in range(3):
        tpl, _ = cut_template(img, m, n, 40 + k, 6.0, affine=True)
        for radius in (0, 2):
            g, dec = S.search(i, tpl, "egs", decision=True, refine_radius=radius, **kw)
            ot = O.te_search(img, tpl, oe["h"], oe["w"], decision=True, radius=radius)
            same_answer(g, ot, "egs")
            same_counts(g, ot, "egs")
            assert np.array_equal(dec, ot["decision"])
    S.unload(i)


# (image rows, cols, seed, beta, template size, parameters, blurred iterates the oracle must accept).  The
# first three keep the conditioning short (at most one blur is worth its cost at the default 0.5% rule);
# the last two keep blurring while the estimated cost rises by less than 15% (accept_xi = -0.15, lambda of
# rho_max = 1), so three blurred iterates are accepted and 87% of the pixels end blurred.
OPTA_CASES = [
    (140, 150, 500, 2.2, 12, dict(blur_kind=1, max_iters=4), 0),
    (140, 150, 501, 2.8, 12, dict(blur_kind=1, max_iters=4), 0),
    (140, 150, 502, 2.8, 12, dict(blur_kind=0, max_iters=4), 0),
    (96, 112, 7102, 3.0, 24, dict(blur_kind=1, rho_max=1.0, accept_xi=-0.15), 3),
    (96, 112, 7102, 3.0, 24, dict(blur_kind=0, rho_max=1.0, accept_xi=-0.15), 3),
]


def _trace(steps):
    return [{k: s[k] for k in ("k", "d", "passes", "reverted", "h", "w", "cost", "accepted")} for s in steps]


@pytest.mark.parametrize("case", OPTA_CASES, ids=[f"opta{k}" for k in range(len(OPTA_CASES))])
def test_opta_parity(S, case):
    """Alg. 3 conditioning for the exact search (every EGS count adds the angle to the original block):
    trace, conditioned image, group size and radius equal the oracle's; every search returns the exhaustive
    answer with the oracle's counts and decision map."""
    p, q, seed, beta, m, kw, min_acc = case
    img = aerial_image(p, q, seed, beta=beta)
    n = m
    print(f"opta parity {p}x{q} seed {seed} m {m} {kw}", flush=True)
    oo = O.opta(img, m, n, **kw)
    assert sum(s["accepted"] for s in oo["trace"][1:]) >= min_acc
    i = S.load(img)
    info = S.prepare(i, m, n, "opta", **kw)
    assert (info["h"], info["w"], info["cost"], info["radius"]) == (oo["h"], oo["w"], oo["cost"], oo["radius"])
    assert _trace(info["opta"]) == _trace(oo["trace"])
    J = S.prep_image(i, m, n)
    assert np.array_equal(J, oo["image"])
    if min_acc:
        assert (J != img).mean() > 0.5
    for k in range(3):
        tpl, _ = cut_template(img, m, n, 70 + k, 8.0, affine=True)
        for extra in (0, 3):
            radius = max(oo["radius"], extra)
            g, dec = S.search(i, tpl, "opta", decision=True, refine_radius=extra, **kw)
            os_ = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], radius, decision=True)
            full = O.full_search(img, tpl)
            same_answer(g, full, "opta vs full")
            same_counts(g, os_, "opta vs oracle opta")
            odec = os_["decision"].copy()
            odec[odec == 1] = 3
            assert np.array_equal(dec, odec)
    S.unload(i)


# Scan 2 bins survivors by tile of 32 x 256 locations.  tile_dense_min 1: every tile with a survivor (and every
# super-tile of four tiles with four) is matched whole on int8 MFMA; -1: survivor by survivor only; 8: a mix;
# 0: the built-in value.  Images span several tile rows and columns with ragged edges; the tall template's
# tiles take the survivor path from global memory (its image region does not fit LDS), the wide one has no
# MFMA path; the 64 x 64 template's tiles split their survivors into parts matched by different blocks.
TILE_CASES = [(300, 700, 24, 24, 25.0, "te_fixed"), (420, 300, 40, 17, 30.0, "egs"), (200, 520, 16, 16, 20.0, "opta"),
              (520, 90, 400, 8, 12.0, "te_fixed"), (150, 600, 20, 150, 20.0, "egs"),
              (230, 600, 64, 64, 30.0, "te_fixed")]


@pytest.mark.parametrize("dense", [1, 8, -1, 0])
@pytest.mark.parametrize("case", TILE_CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}x{c[3]}-{c[5]}" for c in TILE_CASES])
def test_survivor_tile_paths(S, case, dense):
    p, q, m, n, noise, mode = case
    print(f"survivor tiles {case} dense {dense}", flush=True)
    img = aerial_image(p, q, 7000 + p + q, beta=2.2)
    i = S.load(img)
    kw = dict(group_h=3, group_w=3) if mode == "te_fixed" else {}
    for k in range(2):
        tpl, _ = cut_template(img, m, n, 7100 + k, noise, affine=True)
        full = O.full_search(img, tpl)
        for radius in (0, 2):
            g, dec = S.search(i, tpl, mode, decision=(mode != "opta"), refine_radius=radius, tile_dense_min=dense,
                              **kw) if mode != "opta" else (S.search(i, tpl, mode, refine_radius=radius,
                                                                     tile_dense_min=dense), None)
            same_answer(g, full, f"tiles {mode} dense {dense}")
            if mode == "te_fixed":
                ot = O.te_search(img, tpl, 3, 3, decision=True, radius=radius)
            elif mode == "egs":
                info = S.prepare(i, m, n, "egs")
                ot = O.te_search(img, tpl, info["h"], info["w"], decision=True, radius=radius)
            else:
                oo = O.opta(img, m, n)
                ot = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], max(oo["radius"], radius))
            same_counts(g, ot, f"tiles {mode} dense {dense}")
            if dec is not None:
                assert np.array_equal(dec, ot["decision"])
            assert g["n_survivors"] > 0
    S.unload(i)


@pytest.mark.parametrize("dense", [1, -1])
def test_persistent_tile_grids(S, dense):
    """More survivor tiles than the tile kernels' persistent grids hold blocks (2600 x 4200 image, 16 x 16
    template: 1,377 tiles of 32 x 256 locations), so blocks match several tiles in turn, all dense (1) or all
    survivor by survivor (-1): answer, counts and decision map equal the oracle's."""
    print(f"persistent tile grids dense {dense}", flush=True)
    img = aerial_image(2600, 4200, 4242, beta=2.2)
    i = S.load(img)
    tpl, _ = cut_template(img, 16, 16, 4243, 20.0, affine=True)
    full = O.full_search(img, tpl)
    g, dec = S.search(i, tpl, "te_fixed", decision=True, group_h=3, group_w=3, refine_radius=2,
                      tile_dense_min=dense)
    same_answer(g, full, f"persistent tiles dense {dense}")
    ot = O.te_search(img, tpl, 3, 3, decision=True, radius=2)
    same_counts(g, ot, f"persistent tiles dense {dense}")
    assert np.array_equal(dec, ot["decision"])
    assert g["n_survivors"] > 100000
    S.unload(i)


@pytest.mark.parametrize("radius", [3, 5, 9])
def test_large_refinement_windows(S, radius):
    """Refinement windows of 49 to 361 locations (more than one wave's lanes for scan 2's threshold), with
    and without the decision map (the graphed and the eager launch), TE on the original image and OptA on
    the conditioned one: answer, counts and decisions equal the oracle's."""
    img = aerial_image(130, 160, 900 + radius, beta=2.4)
    m = n = 14
    i = S.load(img)
    oo = O.opta(img, m, n, max_iters=3)
    S.prepare(i, m, n, "opta", max_iters=3)
    for k in range(2):
        tpl, _ = cut_template(img, m, n, 1900 + 10 * radius + k, 10.0, affine=True)
        full = O.full_search(img, tpl)
        ot = O.te_search(img, tpl, 3, 4, decision=True, radius=radius)
        for want_dec in (False, True):
            if want_dec:
                g, dec = S.search(i, tpl, "te_fixed", decision=True, group_h=3, group_w=4, refine_radius=radius)
                assert np.array_equal(dec, ot["decision"])
            else:
                for _ in range(3):  # eager, captured, replayed
                    g = S.search(i, tpl, "te_fixed", group_h=3, group_w=4, refine_radius=radius)
                    same_answer(g, full, f"te radius {radius}")
                    same_counts(g, ot, f"te radius {radius}")
            same_answer(g, full, f"te radius {radius}")
            same_counts(g, ot, f"te radius {radius}")
        rad = max(oo["radius"], radius)
        os_ = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], rad, decision=True)
        for _ in range(3):
            g = S.search(i, tpl, "opta", max_iters=3, refine_radius=radius)
            same_answer(g, full, f"opta radius {radius}")
            same_counts(g, os_, f"opta radius {radius}")
    S.unload(i)


@pytest.mark.parametrize("shape", [(6, 300), (3, 520), (40, 260)])
def test_wide_templates(S, shape):
    """Templates wider than 256 pixels (rows of more than 64 words, so the wave dot products take a row in
    several passes): dense search, TE with and without a refinement window, EGS, and Alg. 1 in its direct
    form (large groups), all against the oracle."""
    m, n = shape
    img = aerial_image(110, 720, 4000 + n)
    tpl, _ = cut_template(img, m, n, 4100 + n, 6.0)
    i = S.load(img)
    full = O.full_search(img, tpl)
    same_answer(S.search(i, tpl, "full"), full, f"full {shape}")
    for radius in (0, 2):
        ot = O.te_search(img, tpl, 3, 3, radius=radius)
        g = S.search(i, tpl, "te_fixed", group_h=3, group_w=3, refine_radius=radius)
        same_answer(g, full, f"te {shape} r={radius}")
        same_counts(g, ot, f"te {shape} r={radius}")
    oe = O.egs(img, m, n)
    ge = S.search(i, tpl, "egs")
    same_answer(ge, full, f"egs {shape}")
    assert (ge["group_h"], ge["group_w"]) == (oe["h"], oe["w"])
    if shape == (6, 300):  # OptA: conditioning traces, the conditioned image, the exact search
        oo = O.opta(img, m, n, max_iters=3)
        info = S.prepare(i, m, n, "opta", max_iters=3)
        assert (info["h"], info["w"], info["cost"]) == (oo["h"], oo["w"], oo["cost"])
        assert np.array_equal(S.prep_image(i, m, n), oo["image"])
        go = S.search(i, tpl, "opta", max_iters=3, refine_radius=2)
        os_ = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], max(oo["radius"], 2))
        same_answer(go, full, f"opta {shape}")
        same_counts(go, os_, f"opta {shape}")
    hw = (5, 9) if m * n < 2024 else (9, 9)  # (h w - 1) 46 >= m n: the direct form of Alg. 1
    if (hw[0] * hw[1] - 1) * 46 >= m * n:
        g = Z.zts_debug_autocorr(S.ctx, i, img.shape, m, n, *hw)
        o = O.autocorr(img, m, n, *hw)
        for a_, b_ in zip(g, o):
            assert np.array_equal(a_, b_)
    S.unload(i)


def _sweep_cases():
    rng = np.random.default_rng(20261203)
    out = []
    for k in range(16):
        p, q = int(rng.integers(40, 200)), int(rng.integers(40, 260))
        m, n = int(rng.integers(2, min(p, 48))), int(rng.integers(2, min(q, 140)))
        hw = (int(rng.integers(1, 8)), int(rng.integers(1, 8)))
        radius = int(rng.integers(0, 4))
        out.append((k, p, q, m, n, hw, radius))
    return out


@pytest.mark.parametrize("case", _sweep_cases(), ids=lambda c: "c%d_%dx%d_t%dx%d" % c[:5])
def test_random_sweep(S, case):
    """Seeded random shapes (image, template, group size, refinement radius): TE and the int8-MFMA
    exhaustive search against the oracle, decisions included."""
    k, p, q, m, n, (h, w), radius = case
    img = spectral_image(p, q, float(1.6 + 0.1 * (k % 8)), 7000 + k)
    tpl, _ = cut_template(img, m, n, 7100 + k, 5.0)
    if tpl.min() == tpl.max():
        tpl[0, 0] ^= 1
    print(f"sweep case {case}", flush=True)
    i = S.load(img)
    full = O.full_search(img, tpl)
    ot = O.te_search(img, tpl, h, w, decision=True, radius=radius)
    g, dec = S.search(i, tpl, "te_fixed", decision=True, group_h=h, group_w=w, refine_radius=radius)
    same_answer(g, full, f"te {case}")
    same_counts(g, ot, f"te {case}")
    assert np.array_equal(dec, ot["decision"])
    if n <= 128:
        same_answer(S.search(i, tpl, "full_mfma"), full, f"full_mfma {case}")
    S.unload(i)


@pytest.mark.parametrize("k", range(8))
def test_random_sweep_opta_and_batch(S, k):
    """Seeded random shapes for the prepared modes: EGS and OptA (conditioning traces and the exact search
    with refinement radius 0..2) and one batched call of mixed template sizes, against the oracle."""
    rng = np.random.default_rng(880 + k)
    p, q = int(rng.integers(60, 170)), int(rng.integers(60, 220))
    m, n = int(rng.integers(4, 24)), int(rng.integers(4, 40))
    img = aerial_image(p, q, 8800 + k, beta=float(rng.uniform(1.8, 2.8)))
    tpl, _ = cut_template(img, m, n, 8900 + k, 6.0, affine=bool(k & 1))
    print(f"opta sweep {k}: image {p}x{q} template {m}x{n}", flush=True)
    i = S.load(img)
    full = O.full_search(img, tpl)
    oe = O.egs(img, m, n)
    ge = S.search(i, tpl, "egs")
    same_answer(ge, full, f"egs sweep {k}")
    assert (ge["group_h"], ge["group_w"]) == (oe["h"], oe["w"])
    oo = O.opta(img, m, n, max_iters=3)
    info = S.prepare(i, m, n, "opta", max_iters=3)
    assert (info["h"], info["w"], info["cost"], info["radius"]) == (oo["h"], oo["w"], oo["cost"], oo["radius"])
    assert np.array_equal(S.prep_image(i, m, n), oo["image"])
    radius = int(rng.integers(0, 3))
    go = S.search(i, tpl, "opta", max_iters=3, refine_radius=radius)
    os_ = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], max(oo["radius"], radius))
    same_answer(go, full, f"opta sweep {k}")
    same_counts(go, os_, f"opta sweep {k}")
    sizes = [(int(rng.integers(3, 30)), int(rng.integers(3, 60))) for _ in range(int(rng.integers(2, 9)))]
    tpls = [cut_template(img, a_, b_, 9000 + 10 * k + e, 4.0)[0] for e, (a_, b_) in enumerate(sizes)]
    tpls = [t for t in tpls if t.min() != t.max()]
    for r, t in zip(S.search_batch(i, tpls), tpls):
        same_answer(r, O.full_search(img, t), f"batch sweep {k} {t.shape}")
    S.unload(i)


def test_ties_go_to_smallest_index(S):
    rng = np.random.default_rng(3)
    tile = rng.integers(0, 256, (6, 7), dtype=np.uint8)
    img = np.tile(tile, (12, 12))[:70, :80].copy()
    tpl = img[12:24, 14:28].copy()
    o = O.full_search(img, tpl, maps=True)
    assert (o["rho_map"] == o["rho"]).sum() > 1
    i = S.load(img)
    for mode, kw in [("full", {}), ("te_fixed", dict(group_h=3, group_w=3)), ("egs", {}),
                     ("te_fixed", dict(group_h=5, group_w=4, refine_radius=2))]:
        same_answer(S.search(i, tpl, mode, **kw), o, mode)
    S.unload(i)


def test_errors(S):
    img = spectral_image(40, 40, 2.0, 1)
    i = S.load(img)
    with pytest.raises(Z.ZtsError) as e:
        S.search(i, np.full((5, 5), 7, np.uint8), "full")
    assert e.value.code == -3
    with pytest.raises(Z.ZtsError) as e:
        S.search(i, np.full((5, 5), 7, np.uint8), "egs")
    assert e.value.code == -3
    with pytest.raises(Z.ZtsError) as e:
        S.search(i, np.zeros((41, 5), np.uint8), "full")
    assert e.value.code == -2
    with pytest.raises(Z.ZtsError) as e:
        S.search(i + 99, img[:5, :5], "full")
    assert e.value.code == -4
    S.unload(i)
    with pytest.raises(Z.ZtsError) as e:
        S.search(i, img[:5, :5], "full")
    assert e.value.code == -4
    big = spectral_image(300, 300, 2.0, 2)
    j = S.load(big)
    with pytest.raises(Z.ZtsError) as e:
        S.search(j, big[:129, :129], "full")
    assert e.value.code == -2
    S.unload(j)


def test_device_entry_points_match_host_ones(S):
    import torch
    img = aerial_image(200, 220, 8)
    tpl, _ = cut_template(img, 24, 24, 9, 5.0)
    i = S.load(img)
    j = S.load_device(torch.from_numpy(img).cuda())
    t = torch.from_numpy(tpl).cuda()
    a = S.search(i, tpl, "egs")
    b = Z.zts_search_device(S.ctx, j, t, "egs")
    for k in KEYS + ("n_eliminated", "n_survivors", "n_computed"):
        assert a[k] == b[k]
    # the same call filling a caller's result record, repeatedly (the record is overwritten each time)
    res = Z.Result()
    for _ in range(3):
        out = Z.zts_search_device(S.ctx, j, t, "egs", Z.zts_params_default(), 0, out=res)
        assert out is res
        for k in KEYS + ("n_eliminated", "n_survivors", "n_computed"):
            assert getattr(res, k) == a[k]
    # int8 MFMA from a device template whose rows are strided (a column slice of a wider tensor)
    wide = torch.zeros((24, 40), dtype=torch.uint8, device="cuda")
    wide[:, 5:29] = t
    c = Z.zts_search_device(S.ctx, j, wide[:, 5:29], "full_mfma")
    d = S.search(i, tpl, "full_mfma")
    o = O.full_search(img, tpl)
    for k in KEYS:
        assert c[k] == d[k] == o[k]
    S.unload(i)
    S.unload(j)


def test_workload2_full_size_sampled(S):
    """The named 2048x2048 / 64x64 workload at full size, as the benchmark runs it."""
    w = workload(2)
    img = w["images"][0]
    tpl, loc, _ = w["templates"][0]
    i = S.load(img)
    o = O.full_search(img, tpl)
    assert (o["y"], o["x"]) == loc
    same_answer(S.search(i, tpl, "full"), o, "full")
    oe = O.egs(img, 64, 64)
    info = S.prepare(i, 64, 64, "egs")
    assert info["egs"] == oe["trace"]
    for radius in (0, 2):
        ot = O.te_search(img, tpl, oe["h"], oe["w"], radius=radius)
        g = S.search(i, tpl, "egs", refine_radius=radius)
        same_answer(g, o, "egs")
        same_counts(g, ot, "egs")
    # sampled exact sums at full size
    num, dr, rho32 = Z.zts_debug_full_map(S.ctx, i, img.shape, tpl)
    rng = np.random.default_rng(11)
    Ly, Lx = num.shape
    for _ in range(200):
        y, x = int(rng.integers(0, Ly)), int(rng.integers(0, Lx))
        blk = img[y:y + 64, x:x + 64]
        sub = O.full_search(blk, tpl)
        assert (num[y, x], dr[y, x]) == (sub["num"], sub["den_r"])
        assert abs(rho32[y, x] - sub["rho"]) <= RHO32_TOL
    S.unload(i)


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_mfma_matches_oracle(S, seed):
    """Mixed sizes (several templates per size, a 17-template group, ragged n) in one call."""
    rng = np.random.default_rng(900 + seed)
    img = aerial_image(150, 170, 60 + seed)
    sizes = [(16, 16)] * 17 + [(32, 32)] * 3 + [(20, 36)] * 2 + [(48, 48), (7, 5), (64, 64)]
    tpls = []
    for k, (m, n) in enumerate(sizes):
        t, _ = cut_template(img, m, n, 1000 * seed + k, 6.0)
        tpls.append(t)
    tpls.append(np.full((9, 9), 5, np.uint8))  # flat: per-template error
    i = S.load(img)
    res = S.search_batch(i, tpls)
    for k, t in enumerate(tpls):
        if k == len(tpls) - 1:
            assert res[k]["status"] == -3
            continue
        o = O.full_search(img, t)
        assert res[k]["status"] == 0
        same_answer(res[k], o, f"batch template {k} {t.shape}")
        assert res[k]["n_computed"] == o["n_locations"]
    S.unload(i)


@pytest.mark.parametrize("period", [16, 8, 4])
def test_batch_mfma_ties(S, period):
    """A periodic image: every template matches exactly at many locations, so
    the answer is the smallest-index tie.  16 templates of one size share
    template tiles; the two of another size run one per launch block row.
    Period 16 keeps every block's candidate list within its capacity, period
    8 overflows the single-template lists, period 4 overflows both kinds and
    takes the streaming fallbacks."""
    rng = np.random.default_rng(31 + period)
    base = rng.integers(0, 256, (period, period), dtype=np.uint8)
    img = np.ascontiguousarray(np.tile(base, (300 // period + 1, 600 // period + 1))[:300, :600])
    tpls = []
    for k in range(18):
        m, n = (16, 16) if k < 16 else (24, 40)
        y, x = rng.integers(0, 300 - m), rng.integers(0, 600 - n)
        tpls.append(np.ascontiguousarray(img[y:y + m, x:x + n]))
    i = S.load(img)
    res = S.search_batch(i, tpls)
    for k, t in enumerate(tpls):
        o = O.full_search(img, t)
        same_answer(res[k], o, f"periodic {period} template {k}")
    S.unload(i)


def test_batch_mfma_flat_regions(S):
    """Flat image regions (rho := 0 there): a fully flat image, where every
    location ties at 0, and an image flat on its left half."""
    rng = np.random.default_rng(77)
    flat = np.full((120, 400), 93, np.uint8)
    half = aerial_image(120, 400, 5)
    half[:, :200] = 40
    for img in (flat, half):
        tpls = [cut_template(aerial_image(120, 400, 6), 16, 16, k, 4.0)[0] for k in range(16)]
        tpls += [cut_template(aerial_image(120, 400, 6), 20 + k, 12 + 3 * k, 50 + k, 4.0)[0] for k in range(3)]
        tpls.append(np.ascontiguousarray(img[10:42, 180:212]))  # flat on the flat image
        i = S.load(img)
        res = S.search_batch(i, tpls)
        for k, t in enumerate(tpls):
            if t.min() == t.max():
                assert res[k]["status"] == -3
                continue
            o = O.full_search(img, t)
            same_answer(res[k], o, f"flat-region template {k}")
        S.unload(i)


# The paper's OptA (Alg. 3 as printed: EGS on each blurred image alone) on inputs where it accepts two or
# three blurred iterates and grows the groups from 3x3 to 5x5, plus the short-conditioning inputs above.
PAPER_CASES = [
    (96, 96, 7002, 2.6, 24, dict(blur_kind=1, rho_max=1.0), 3),
    (96, 96, 7002, 2.6, 24, dict(blur_kind=0, rho_max=1.0), 3),
    (128, 128, 7001, 2.6, 24, dict(blur_kind=1, rho_max=1.0), 2),
    (140, 150, 500, 2.2, 12, dict(blur_kind=1, max_iters=4), 0),
    (140, 150, 502, 2.8, 12, dict(blur_kind=0, max_iters=4), 0),
]


@pytest.mark.parametrize("case", PAPER_CASES, ids=[f"paper{k}" for k in range(len(PAPER_CASES))])
def test_opta_paper_parity(S, case):
    """The paper's own OptA against the oracle's: the conditioning trace, conditioned image, group size and
    radius, then the same answer (the localisation window's best on I around the conditioned image's best)
    and the same counts.  The share of answers equal to the exhaustive one, and within 4 px of it, is
    printed (the search is inexact by design)."""
    p, q, seed, beta, m, kw, min_acc = case
    n = m
    img = aerial_image(p, q, seed, beta=beta)
    print(f"paper opta parity {p}x{q} seed {seed} m {m} {kw}", flush=True)
    oo = O.opta(img, m, n, paper=True, **kw)
    acc = [s for s in oo["trace"] if s["accepted"]]
    assert len(acc) - 1 >= min_acc
    if min_acc:
        assert len({s["h"] for s in acc}) >= 2  # the groups grew across iterations
    i = S.load(img)
    info = S.prepare(i, m, n, "opta_paper", **kw)
    assert (info["h"], info["w"], info["cost"], info["radius"]) == (oo["h"], oo["w"], oo["cost"], oo["radius"])
    assert _trace(info["opta"]) == _trace(oo["trace"])
    last = O.egs(oo["image"], m, n, h0=acc[-2]["h"] if len(acc) > 1 else 3, w0=acc[-2]["w"] if len(acc) > 1 else 3)
    if len(acc) > 1:
        assert info["egs"] == last["trace"]
    J = S.prep_image(i, m, n, "opta_paper")
    assert np.array_equal(J, oo["image"])
    exact = near = total = 0
    for k in range(4):
        tpl, _ = cut_template(img, m, n, 70 + k, 8.0, affine=True)
        full = O.full_search(img, tpl)
        for extra in (0, 3):
            radius = max(oo["radius"], extra)
            g = S.search(i, tpl, "opta_paper", refine_radius=extra, **kw)
            o = O.opta_paper_search(img, oo["image"], tpl, oo["h"], oo["w"], radius)
            same_answer(g, o, f"paper opta seed {seed} tpl {k} r {radius}")
            for key in ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed"):
                assert g[key] == o[key], (key, g[key], o[key])
            total += 1
            exact += (g["y"], g["x"]) == (full["y"], full["x"])
            near += abs(g["y"] - full["y"]) <= 4 and abs(g["x"] - full["x"]) <= 4
    print(f"  paper OptA: {exact}/{total} exact, {near}/{total} within 4 px", flush=True)
    S.unload(i)


# Images at the 32767-pixel dimension limit and templates of the 16384-pixel limit in four aspect
# ratios.  `refuse` lists the modes whose kernels cannot stage the shape in one workgroup's LDS
# (ZTS_FULL stages 31 + m image rows of the template's width, the eliminating modes the whole
# template in 16-byte rows, ZTS_FULL_MFMA takes n <= 128): they return ZTS_E_SIZE before launching.
MAX_CASES = [
    ("wide image", 24, 32767, 8, 8, set()),
    ("tall image", 32767, 24, 8, 8, set()),
    ("128x128 template", 180, 200, 128, 128, set()),
    ("1x16384 template", 4, 16400, 1, 16384, {"full", "full_mfma"}),
    ("2048x8 template", 2100, 40, 2048, 8, {"full"}),
    ("16384x1 template", 16400, 4, 16384, 1, {"full", "te_fixed", "egs", "opta"}),
]


@pytest.mark.parametrize("case", MAX_CASES, ids=[c[0] for c in MAX_CASES])
def test_maximum_sizes(S, case):
    """Every mode either returns the oracle's exact answer (counts covering every location, TE's
    counts equal to the oracle's) or refuses the shape with ZTS_E_SIZE."""
    name, p, q, m, n, refuse = case
    print(f"maximum sizes: {name} ({p}x{q} image, {m}x{n} template)", flush=True)
    img = spectral_image(p, q, 2.0, 77)
    tpl, _ = cut_template(img, m, n, 78, 5.0)
    full = O.full_search(img, tpl)
    L = (p - m + 1) * (q - n + 1)
    i = S.load(img)
    for mode, kw in [("full", {}), ("full_mfma", {}), ("te_fixed", dict(group_h=3, group_w=3)), ("egs", {}),
                     ("opta", dict(refine_radius=2))]:
        print(f"  {mode}", flush=True)
        if mode in refuse:
            with pytest.raises(Z.ZtsError) as e:
                S.search(i, tpl, mode, **kw)
            assert e.value.code == -2, (name, mode)
            continue
        g = S.search(i, tpl, mode, **kw)
        same_answer(g, full, f"{name} {mode}")
        assert g["n_computed"] + g["n_eliminated"] == g["n_locations"] == L, (name, mode)
        if mode == "te_fixed":
            same_counts(g, O.te_search(img, tpl, 3, 3, decision=False, radius=-1), f"{name} te")
    S.unload(i)
    if name == "wide image":  # one column more than the limit
        with pytest.raises(Z.ZtsError) as e:
            S.load(np.zeros((1, 32768), np.uint8))
        assert e.value.code == -2


@pytest.mark.parametrize("mode", ["te_fixed", "egs", "opta"])
def test_detection_floor(S, mode):
    """rho_floor with floor_prune: scan 2 eliminates against max(best0, floor).  Answers, counts and decisions
    equal the oracle's searches with the same floor; above_floor says whether rho reaches the floor; with the
    floor at or below the true maximum the answer is the exhaustive one.  Without floor_prune the floor only
    labels the exhaustive answer.  A noise template (no true match) is included."""
    from synth import noise_template
    img = aerial_image(180, 210, 4321, beta=2.2)
    m = n = 14
    i = S.load(img)
    kw = dict(group_h=3, group_w=3) if mode == "te_fixed" else {}
    info = S.prepare(i, m, n, mode, **kw) if mode != "te_fixed" else {"h": 3, "w": 3}
    oo = O.opta(img, m, n) if mode == "opta" else None
    tpls = [cut_template(img, m, n, 4400 + k, 10.0, affine=True)[0] for k in range(2)] + [noise_template(m, n, 4500)]
    for k, tpl in enumerate(tpls):
        full = O.full_search(img, tpl)
        for fl in (full["rho"] - 0.05, full["rho"], 0.9, 0.999):
            print(f"floor {mode} template {k} floor {fl:.4f}", flush=True)
            if mode == "opta":
                o = O.opta_search(img, oo["image"], tpl, oo["h"], oo["w"], oo["radius"], decision=False, floor=fl)
            else:
                o = O.te_search(img, tpl, info["h"], info["w"], decision=True, floor=fl)
            if mode == "opta":
                g = S.search(i, tpl, mode, rho_floor=fl, floor_prune=1)
            else:
                g, dec = S.search(i, tpl, mode, decision=True, rho_floor=fl, floor_prune=1, **kw)
                assert np.array_equal(dec, o["decision"])
            same_counts(g, o, f"floor {fl}")
            assert g["above_floor"] == int(g["rho"] >= fl)
            if fl <= full["rho"]:
                same_answer(g, o, f"floor {fl}")
                same_answer(g, full, "floor at or below the maximum")
            else:
                # below the floor nothing is claimed but that the answer is an attained location at least as
                # good as the best centre or survivor (dense tiles may also have matched eliminated locations)
                y, x = g["y"], g["x"]
                at = O.full_search(img[y:y + m, x:x + n], tpl)
                assert (g["num"], g["den_t"], g["den_r"], g["rho"]) == (at["num"], at["den_t"], at["den_r"], at["rho"])
                assert g["rho"] >= o["rho"] and g["above_floor"] == 0
            lab = S.search(i, tpl, mode, rho_floor=fl, **kw)
            same_answer(lab, full, "floor as a label")
            assert lab["above_floor"] == int(full["rho"] >= fl)
    S.unload(i)


@pytest.mark.parametrize("mode,kw", [("te_fixed", dict(group_h=3, group_w=4)), ("egs", dict(refine_radius=2)),
                                     ("opta", dict(refine_radius=2)), ("opta", {}), ("opta_paper", {})])
def test_batch_pruned_equals_single_searches(S, mode, kw):
    """zts_search_batch_pruned: templates of several sizes (groups of 1, 3 and 6 templates, so scan 1 runs for
    4 + 2 templates in one launch, and a width over 128 that has no MFMA scan 1), a flat template, in one call;
    every result equals the single search's (location, integers, binary64 rho, counts) and, for the exact
    modes, the oracle's plain answer."""
    img = aerial_image(220, 260, 5150, beta=2.3)
    sizes = [(24, 24)] * 6 + [(17, 29)] * 3 + [(40, 40), (12, 140)]
    tpls = [cut_template(img, m, n, 5200 + k, 9.0, affine=True)[0] for k, (m, n) in enumerate(sizes)]
    tpls.insert(4, np.full((24, 24), 77, np.uint8))  # flat: its own status, the others unaffected
    i = S.load(img)
    res = S.search_batch_pruned(i, tpls, mode, **kw)
    assert len(res) == len(tpls)
    for k, t in enumerate(tpls):
        print(f"batch pruned {mode} template {k} {t.shape}", flush=True)
        if t.min() == t.max():
            assert res[k]["status"] == -3
            continue
        g = S.search(i, t, mode, **kw)
        assert res[k]["status"] == 0
        for key in KEYS + ("rho32", "n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed",
                           "group_h", "group_w", "best0", "n_dense", "n_sparse"):
            assert res[k][key] == g[key], (mode, k, key, res[k][key], g[key])
        if mode != "opta_paper":
            same_answer(res[k], O.full_search(img, t), f"batch pruned {mode} {k}")
    # the device form: the same templates read in place from device memory (one with strided rows)
    import torch
    tdev = [torch.from_numpy(t).cuda() for t in tpls]
    wide = torch.zeros((24, 40), dtype=torch.uint8, device="cuda")
    wide[:, 3:27] = tdev[0]
    tdev[0] = wide[:, 3:27]
    out = Z.zts_search_batch_pruned_device(S.ctx, i, Z.DeviceBatch(tdev), mode, Z.zts_params_default(**kw))
    for k in range(len(tpls)):
        d = out[k].as_dict()
        for key in KEYS + ("status", "n_eliminated", "n_survivors", "n_computed"):
            assert d[key] == res[k][key], (mode, k, key)
    S.unload(i)
