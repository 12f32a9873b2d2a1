"""Pins for the CPU oracle against things other than itself.

Each test checks the oracle against the paper's printed numbers, a closed
form, a library routine (numpy, scipy), an invariant, or brute force on tiny
inputs, so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails here.  CPU only.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

import oracle as O
from synth import spectral_image, aerial_image, cut_template

RNG = np.random.default_rng(20240601)


def tiny_image(p, q, seed, kind="spectral"):
    rng = np.random.default_rng(seed)
    if kind == "spectral":
        return spectral_image(p, q, 2.0, seed)
    if kind == "uniform":
        return rng.integers(0, 256, (p, q), dtype=np.uint8)
    if kind == "flat_patches":
        img = spectral_image(p, q, 2.0, seed)
        img[: p // 2, : q // 2] = 200
        return img
    if kind == "periodic":
        tile = rng.integers(0, 256, (4, 5), dtype=np.uint8)
        return np.tile(tile, (p // 4 + 1, q // 5 + 1))[:p, :q].copy()
    raise ValueError(kind)


# ---------------------------------------------------------------- Eq. 1

def test_canonical_rho_matches_literal_two_pass():
    for k in range(200):
        m, n = int(RNG.integers(1, 12)), int(RNG.integers(1, 12))
        a = RNG.integers(0, 256, (m, n), dtype=np.uint8)
        b = RNG.integers(0, 256, (m, n), dtype=np.uint8)
        if k % 7 == 0:
            b = np.clip(a.astype(int) * 2 + 3, 0, 255).astype(np.uint8)
        mn = m * n
        sa, sb = int(a.sum(dtype=np.int64)), int(b.sum(dtype=np.int64))
        da = mn * int((a.astype(np.int64) ** 2).sum()) - sa * sa
        db = mn * int((b.astype(np.int64) ** 2).sum()) - sb * sb
        num = mn * int((a.astype(np.int64) * b).sum()) - sa * sb
        r = O.rho(num, da, db)
        assert abs(r - O.rho_twopass(a, b)) <= 1e-12
        assert -1.0 - 1e-15 <= r <= 1.0 + 1e-15
        if da and db:
            s = O.sin(num, da, db)
            assert abs(r * r + s * s - 1.0) <= 1e-12
            assert abs(s - math.sqrt(max(0.0, 1.0 - r * r))) <= 1e-7


def test_full_search_maps_match_numpy_corrcoef_and_scipy():
    img = tiny_image(24, 29, 3)
    tpl = img[5:12, 9:17].copy()
    tpl[0, 0] ^= 0x55
    res = O.full_search(img, tpl, maps=True)
    m, n = tpl.shape
    xs = scipy.signal.correlate2d(img.astype(np.int64), tpl.astype(np.int64), mode="valid")
    assert np.array_equal(res["xs_map"], xs)
    Ly, Lx = res["rho_map"].shape
    for y in range(Ly):
        for x in range(Lx):
            blk = img[y:y + m, x:x + n].astype(np.float64).ravel()
            ref = np.corrcoef(tpl.astype(np.float64).ravel(), blk)[0, 1]
            assert abs(res["rho_map"][y, x] - ref) <= 1e-12
    flat = res["rho_map"].ravel()
    best = int(np.argmax(flat))
    assert (res["y"], res["x"]) == divmod(best, Lx)
    assert res["rho"] == flat[best]


def test_location_stats_running_sums_equal_direct_loops():
    for seed in range(5):
        img = tiny_image(19, 23, seed, "uniform")
        for (m, n) in [(1, 1), (3, 5), (7, 4), (19, 23)]:
            a = O.location_stats(img, m, n)
            b = O.location_stats(img, m, n, running_sums=True)
            for u, v in zip(a, b):
                assert np.array_equal(u, v)
            S, S2, D = a
            assert (D >= 0).all()


def test_noise_free_cut_gives_rho_one():
    img = tiny_image(40, 40, 11)
    y0, x0, m, n = 13, 7, 9, 11
    tpl = img[y0:y0 + m, x0:x0 + n].copy()
    r = O.full_search(img, tpl)
    assert (r["y"], r["x"]) == (y0, x0)
    assert r["num"] == r["den_t"] == r["den_r"]
    assert abs(r["rho"] - 1.0) <= 2 * np.finfo(np.float64).eps


def test_affine_intensity_invariance():
    img = (tiny_image(36, 36, 5).astype(np.int64) // 4).astype(np.uint8)  # values <= 63
    tpl = img[10:18, 4:14].copy()
    tpl[3, 3] = 17
    a, b = 3, 20
    tpl2 = (a * tpl.astype(np.int64) + b).astype(np.uint8)  # <= 209, no clipping
    r1 = O.full_search(img, tpl, maps=True)
    r2 = O.full_search(img, tpl2, maps=True)
    assert np.array_equal(r2["num_map"], a * r1["num_map"])
    assert r2["den_t"] == a * a * r1["den_t"]
    assert np.abs(r2["rho_map"] - r1["rho_map"]).max() <= 1e-12
    assert (r1["y"], r1["x"]) == (r2["y"], r2["x"])


def test_degenerate_template_is_an_error_and_flat_window_has_rho_zero():
    img = tiny_image(20, 20, 2)
    with pytest.raises(O.OracleError):
        O.full_search(img, np.full((4, 4), 9, np.uint8))
    img[0:6, 0:6] = 77
    tpl = tiny_image(20, 20, 9)[:5, :5].copy()
    r = O.full_search(img, tpl, maps=True)
    assert r["rho_map"][0, 0] == 0.0 and r["dr_map"][0, 0] == 0


# ---------------------------------------------------------------- Eq. 2-4

def test_fig2_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "fig2_bounds.json")))
    lb, ub = O.transitive_bounds(g["rho_a"], g["rho_b"])
    assert round(lb, g["decimals"]) == g["lower"]
    assert round(ub, g["decimals"]) == g["upper"]
    # the pair as printed does not reproduce the printed interval (reading R1)
    lb2, ub2 = O.transitive_bounds(g["rho_a"], g["printed_rho_b"])
    assert round(ub2, 3) != g["upper"]


def test_transitive_gap_and_angle_form():
    for _ in range(500):
        a, b = RNG.uniform(-1, 1, 2)
        lb, ub = O.transitive_bounds(a, b)
        assert abs((ub - lb) - O.transitive_gap(a, b)) <= 1e-14
        A, B = math.acos(a), math.acos(b)
        assert abs(ub - math.cos(A - B)) <= 1e-12
        assert abs(lb - math.cos(A + B)) <= 1e-12


def test_general_bound_is_cosine_of_angle_triangle():
    for _ in range(2000):
        A, B, Cc = RNG.uniform(0, math.pi, 3)
        ok, ub = O.ub_general(math.cos(A), math.sin(A), math.cos(B), math.sin(B), math.cos(Cc), math.sin(Cc))
        gap = abs(A - B) - Cc
        if abs(gap) < 1e-9:
            continue
        assert ok == (gap > 0)
        if ok:
            assert abs(ub - math.cos(gap)) <= 1e-12
    # C = 0 reduces exactly to Eq. 2's canonical form rho_a*rho_b + s_a*s_b
    for _ in range(500):
        ra, rb = RNG.uniform(-1, 1, 2)
        sa, sb = math.sqrt(1 - ra * ra), math.sqrt(1 - rb * rb)
        ok, ub = O.ub_general(ra, sa, rb, sb, 1.0, 0.0)
        if ok:
            assert ub == ra * rb + sa * sb


def _all_blocks(img, m, n):
    p, q = img.shape
    return [img[y:y + m, x:x + n] for y in range(p - m + 1) for x in range(q - n + 1)]


def _exact(a, b):
    a = a.astype(np.int64).ravel()
    b = b.astype(np.int64).ravel()
    mn = a.size
    num = mn * int(a @ b) - int(a.sum()) * int(b.sum())
    da = mn * int(a @ a) - int(a.sum()) ** 2
    db = mn * int(b @ b) - int(b.sum()) ** 2
    return num, da, db


def test_transitive_bounds_hold_on_every_triple_of_blocks():
    img = tiny_image(11, 12, 21, "uniform")
    tpl = tiny_image(4, 4, 22, "uniform")
    blocks = _all_blocks(img, 4, 4)
    rs = {}
    def pair(a, b, key):
        if key not in rs:
            n, da, db = _exact(a, b)
            rs[key] = (O.rho(n, da, db), O.sin(n, da, db), da and db)
        return rs[key]
    count = 0
    for i, c in enumerate(blocks):
        rtc, stc, ok1 = pair(tpl, c, ("t", i))
        for j, o in enumerate(blocks):
            rco, sco, ok2 = pair(c, o, (i, j))
            rto, _, ok3 = pair(tpl, o, ("t", j))
            if not (ok1 and ok2 and ok3):
                continue
            lb, ub = O.transitive_bounds(rtc, rco)
            assert lb - 1e-12 <= rto <= ub + 1e-12
            ok, ub2 = O.ub_general(rtc, stc, rco, sco, 1.0, 0.0)
            if ok:
                assert abs(ub2 - ub) <= 1e-9
                assert rto <= ub2 + 1e-12
            count += 1
    assert count > 5000


def test_composite_bound_holds_through_a_blurred_image():
    """angle(t,o) >= |angle(t,c') - angle(c',o')| - angle(o',o) on all blocks."""
    I = tiny_image(12, 12, 31)
    taps, _ = O.gauss_taps(1.0)
    J = O.blur(I, taps)
    tpl = tiny_image(5, 5, 32, "uniform")
    bi = _all_blocks(I, 5, 5)
    bj = _all_blocks(J, 5, 5)
    checked = 0
    for ci, c in enumerate(bj):
        n, da, db = _exact(tpl, c)
        if not (da and db):
            continue
        ra, sa = O.rho(n, da, db), O.sin(n, da, db)
        for oi in range(len(bi)):
            n2, d2a, d2b = _exact(c, bj[oi])
            n3, d3a, d3b = _exact(bj[oi], bi[oi])
            n4, d4a, d4b = _exact(tpl, bi[oi])
            if not (d2a and d2b and d3a and d3b and d4b):
                continue
            ok, ub = O.ub_general(ra, sa, O.rho(n2, d2a, d2b), O.sin(n2, d2a, d2b), O.rho(n3, d3a, d3b),
                                  O.sin(n3, d3a, d3b))
            rto = O.rho(n4, d4a, d4b)
            if ok:
                assert rto <= ub + 1e-12
                checked += 1
    assert checked > 1000


# ---------------------------------------------------------------- grouping, Alg. 1

def test_group_centre_rule():
    # Ly = 7 with h = 3: rows {0,1,2} {3,4,5} {6}: centres 1, 4, 6
    assert [O.centre_of(7, 1, 3, 1, y) for y in range(7)] == [1, 1, 1, 4, 4, 4, 6]
    # h = 4: rows {0..3} {4,5,6}: centres 1, 5
    assert [O.centre_of(7, 1, 4, 1, y) for y in range(7)] == [1, 1, 1, 1, 5, 5, 5]
    # 2-D: Lx = 5, w = 2: columns {0,1} {2,3} {4}: centres 0, 2, 4
    assert [O.centre_of(1, 5, 1, 2, x) for x in range(5)] == [0, 0, 2, 2, 4]
    assert O.group_count(7, 5, 3, 2) == 3 * 3


@pytest.mark.parametrize("p,q,m,n,h,w", [(14, 17, 3, 4, 3, 3), (15, 15, 5, 5, 4, 2), (20, 13, 6, 3, 5, 5),
                                         (9, 9, 9, 9, 3, 3), (12, 16, 2, 7, 1, 1), (18, 18, 4, 4, 7, 6)])
def test_lsa_running_sums_equal_direct_dot_products(p, q, m, n, h, w):
    for seed in range(3):
        img = tiny_image(p, q, 100 + seed, ["uniform", "spectral", "flat_patches"][seed])
        a = O.autocorr(img, m, n, h, w, method="lsa", nthreads=3)
        b = O.autocorr(img, m, n, h, w, method="direct")
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    # the pairing itself, against blocks cut with numpy and a hand-written tiling
    Ly, Lx = p - m + 1, q - n + 1
    for l in range(0, Ly * Lx, 3):
        y, x = divmod(l, Lx)
        gy, gx = (y // h) * h, (x // w) * w
        cy = gy + (min(h, Ly - gy) - 1) // 2
        cx = gx + (min(w, Lx - gx) - 1) // 2
        n_, dc_, do_ = _exact(img[cy:cy + m, cx:cx + n], img[y:y + m, x:x + n])
        assert (a[0][l], a[1][l], a[2][l]) == (n_, dc_, do_)


# ---------------------------------------------------------------- elimination search

CASES = [(20, 22, 4, 5, 3, 3), (25, 25, 6, 6, 5, 5), (16, 30, 3, 3, 2, 4), (12, 12, 12, 12, 3, 3),
         (30, 21, 7, 4, 4, 3), (18, 18, 5, 5, 1, 1), (28, 28, 8, 8, 9, 9)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("kind", ["spectral", "uniform", "flat_patches", "periodic"])
@pytest.mark.parametrize("radius", [0, 2])
def test_te_search_equals_full_search(case, kind, radius):
    p, q, m, n, h, w = case
    img = tiny_image(p, q, hash((case, kind)) % 1000, kind)
    rng = np.random.default_rng(hash((case, kind, 1)) % 1000)
    y0, x0 = int(rng.integers(0, p - m + 1)), int(rng.integers(0, q - n + 1))
    tpl = np.clip(img[y0:y0 + m, x0:x0 + n].astype(int) + rng.integers(-6, 7, (m, n)), 0, 255).astype(np.uint8)
    if tpl.std() == 0:
        tpl[0, 0] ^= 1
    full = O.full_search(img, tpl, maps=True)
    te = O.te_search(img, tpl, h, w, decision=True, radius=radius)
    for k in ("y", "x", "rho", "num", "den_t", "den_r"):
        assert te[k] == full[k], k
    L = full["rho_map"].size
    dec = te["decision"].ravel()
    rho = full["rho_map"].ravel()
    assert te["n_locations"] == L
    assert te["n_computed"] + te["n_eliminated"] == L
    assert te["n_centres"] == O.group_count(p - m + 1, q - n + 1, h, w)
    assert (dec == 0).sum() == te["n_eliminated"]
    # every eliminated location is strictly below the threshold actually used
    assert (rho[dec == 0] < te["best0"]).all()
    if h == 1 and w == 1:
        assert te["n_eliminated"] == 0


def test_te_search_ties_go_to_smallest_index():
    # a periodic image holds exact duplicates of the best block
    img = tiny_image(24, 24, 7, "periodic")
    tpl = img[8:14, 10:16].copy()
    full = O.full_search(img, tpl, maps=True)
    rho = full["rho_map"].ravel()
    tied = np.flatnonzero(rho == rho.max())
    assert len(tied) > 1
    Lx = full["rho_map"].shape[1]
    assert (full["y"], full["x"]) == divmod(int(tied[0]), Lx)
    for h, w in [(3, 3), (4, 5)]:
        te = O.te_search(img, tpl, h, w)
        assert (te["y"], te["x"]) == (full["y"], full["x"])


# ---------------------------------------------------------------- EGS

def test_egs_threshold_closed_form_and_trace():
    assert abs(math.sqrt(1.0 - 0.8 * 0.8) - 0.6) <= 1e-15
    img = aerial_image(96, 96, 5, beta=2.0)
    m = n = 16
    e = O.egs(img, m, n)
    Ly = Lx = 96 - 16 + 1
    thr = math.sqrt(1.0 - 0.8 * 0.8)
    prev = m * n * Ly * Lx
    for step in e["trace"]:
        h, w = step["h"], step["w"]
        assert step["cc"] == O.group_count(Ly, Lx, h, w)
        num, dc, do = O.autocorr(img, m, n, h, w, method="direct")
        cr = 0
        for l in range(Ly * Lx):
            if O.centre_of(Ly, Lx, h, w, l) == l:
                continue
            if dc[l] == 0 or do[l] == 0 or O.rho(num[l], dc[l], do[l]) < thr:
                cr += 1
        assert step["cr"] == cr
        assert step["ct"] == m * n * (step["cc"] + cr)
        assert step["accepted"] == ((prev - step["ct"]) > 0.005 * prev)
        if step["accepted"]:
            prev = step["ct"]
    assert e["cost"] == prev


def test_egs_one_by_one_group_costs_a_full_search():
    img = tiny_image(30, 30, 3)
    e = O.egs(img, 6, 6, h0=1, w0=1, dh=2, dw=2)
    first = e["trace"][0]
    L = 25 * 25
    assert (first["h"], first["w"], first["cc"], first["cr"]) == (1, 1, L, 0)
    assert first["ct"] == 36 * L and not first["accepted"]
    assert (e["h"], e["w"]) == (1, 1)


# ---------------------------------------------------------------- blur

def test_gaussian_taps():
    for sigma in [0.3, 0.5, 0.5 * math.sqrt(3), 1.0, 0.5 * math.sqrt(7), 1.5, 0.5 * math.sqrt(11), 2.7]:
        taps, d = O.gauss_taps(sigma)
        assert d == math.ceil(3 * sigma)
        assert taps.sum() == 256
        assert np.array_equal(taps, taps[::-1])
        assert (np.diff(taps[d:]) <= 0).all()
        g = np.exp(-np.arange(-d, d + 1) ** 2 / (2 * sigma * sigma))
        assert np.abs(taps - 256 * g / g.sum()).max() <= 1.0
    taps, d = O.gauss_taps(0.0)
    assert d == 0 and list(taps) == [256]


def test_blur_pins(golden_dir):
    params = json.load(open(os.path.join(golden_dir, "paper_parameters.json")))
    W = np.array(params["W"])
    assert np.allclose(O.PAPER_W / O.PAPER_W.sum(), W, atol=0, rtol=1e-15)
    img = tiny_image(33, 41, 8, "uniform")
    # identity
    assert np.array_equal(O.blur(img, np.array([256], np.int32)), img)
    assert np.array_equal(O.blur(img, np.array([1], np.int32)), img)
    # a constant image stays constant
    const = np.full((17, 19), 123, np.uint8)
    for taps in [O.PAPER_W, O.gauss_taps(1.3)[0]]:
        assert (O.blur(const, taps) == 123).all()
    for taps in [O.PAPER_W, O.gauss_taps(0.5)[0], O.gauss_taps(1.5 * math.sqrt(5) / 3)[0], O.gauss_taps(2.2)[0]]:
        out = O.blur(img, taps)
        # reflection symmetry
        assert np.array_equal(O.blur(img[::-1, ::-1].copy(), taps), out[::-1, ::-1])
        # exact against scipy's separable float correlation with nearest-edge borders
        t = taps.astype(np.float64)
        V = scipy.ndimage.correlate1d(img.astype(np.float64), t, axis=1, mode="nearest")
        V = scipy.ndimage.correlate1d(V, t, axis=0, mode="nearest")
        T = float(taps.sum()) ** 2
        ref = np.floor((V + T / 2) / T).astype(np.int64)
        assert np.array_equal(out.astype(np.int64), ref)
        # and within one grey level of the unquantised Gaussian
        if len(taps) > 5 or taps.sum() == 256:
            pass
    sig = 1.2
    taps, d = O.gauss_taps(sig)
    ideal = scipy.ndimage.gaussian_filter(img.astype(np.float64), sig, mode="nearest", truncate=d / sig)
    assert np.abs(O.blur(img, taps).astype(np.float64) - ideal).max() <= 2.0


# ---------------------------------------------------------------- Eq. 28 and revert

def test_lambda_closed_form():
    for rmax, expect in [(1.0, 0.8), (0.95, 0.947350), (0.90, 0.981534)]:
        lam = O.lambda_(0.8, rmax)
        assert abs(lam - math.cos(math.acos(0.8) - math.acos(rmax))) <= 1e-15
        assert round(lam, 6) == expect


def test_revert_fixpoint_invariants():
    I = aerial_image(48, 52, 12, beta=2.0)
    I[5:20, 30:45] = 230
    m = n = 8
    lam = O.lambda_(0.8, 0.95)
    taps, _ = O.gauss_taps(1.5)
    J0 = O.blur(I, taps)
    J, passes, rev = O.revert(I, J0, m, n, lam)
    assert passes >= 1 and rev > 0
    changed = J != J0
    assert np.array_equal(J[changed], I[changed])
    num, dj, di = O.blurcorr(I, J, m, n)
    Ly, Lx = 48 - m + 1, 52 - n + 1
    for l in range(Ly * Lx):
        y, x = divmod(l, Lx)
        if dj[l] == 0 or di[l] == 0:
            assert np.array_equal(J[y:y + m, x:x + n], I[y:y + m, x:x + n])
        else:
            assert O.rho(num[l], dj[l], di[l]) >= lam
    J2, passes2, rev2 = O.revert(I, J, m, n, lam)
    assert passes2 == 0 and rev2 == 0 and np.array_equal(J2, J)


def test_blurcorr_matches_direct_blocks():
    I = tiny_image(15, 17, 4, "uniform")
    J = O.blur(I, O.PAPER_W)
    num, dj, di = O.blurcorr(I, J, 4, 6)
    Lx = 17 - 6 + 1
    for l in range(len(num)):
        y, x = divmod(l, Lx)
        n_, a_, b_ = _exact(J[y:y + 4, x:x + 6], I[y:y + 4, x:x + 6])
        assert (num[l], dj[l], di[l]) == (n_, a_, b_)


# ---------------------------------------------------------------- OptA

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_opta_search_equals_full_search(seed):
    I = aerial_image(64, 64, 40 + seed, beta=2.6 if seed else 2.0)
    m = n = 12
    op = O.opta(I, m, n, nthreads=4)
    tr = op["trace"]
    assert tr[0]["k"] == 0
    for a, b in zip(tr[:-1], tr[1:]):
        if b["accepted"]:
            assert (a["cost"] - b["cost"]) > 0.005 * b["cost"]
            assert b["h"] >= a["h"]
    for radius in [op["radius"], 3]:
        for k in range(3):
            tpl, _ = cut_template(I, m, n, 500 + 10 * seed + k, 6.0)
            full = O.full_search(I, tpl)
            s = O.opta_search(I, op["image"], tpl, op["h"], op["w"], radius, decision=True)
            for key in ("y", "x", "rho", "num", "den_t", "den_r"):
                assert s[key] == full[key]
            assert s["n_computed"] + s["n_eliminated"] == s["n_locations"]


def test_opta_search_with_a_forced_blur_is_exact():
    """A blurred image that OptA would not accept still gives the exact answer."""
    I = aerial_image(60, 70, 9, beta=2.2)
    m, n = 10, 9
    taps, _ = O.gauss_taps(1.0)
    J, _, _ = O.revert(I, O.blur(I, taps), m, n, O.lambda_(0.8, 0.95))
    for k in range(4):
        tpl, _ = cut_template(I, m, n, 900 + k, 8.0, affine=True)
        full = O.full_search(I, tpl)
        for (h, w, r) in [(3, 3, 0), (5, 5, 2), (4, 6, 1)]:
            s = O.opta_search(I, J, tpl, h, w, r)
            assert (s["y"], s["x"], s["rho"]) == (full["y"], full["x"], full["rho"])


def test_window_search_is_the_full_map_restricted_to_the_window():
    """Section IV-C's localisation stage against the full map: every window location's rho is the map's,
    the best is the window slice's argmax with ties to the smallest index, clipped at the grid edges."""
    img = aerial_image(50, 61, 17, beta=2.4)
    tpl, _ = cut_template(img, 9, 11, 4, 6.0)
    f = O.full_search(img, tpl, maps=True)
    R = f["rho_map"]
    Ly, Lx = R.shape
    for cy, cx, r in [(20, 20, 2), (0, 0, 3), (Ly - 1, Lx - 1, 4), (f["y"], f["x"], 0), (10, Lx - 2, 8)]:
        w = O.window_search(img, tpl, cy, cx, r)
        y0, y1, x0, x1 = max(0, cy - r), min(Ly, cy + r + 1), max(0, cx - r), min(Lx, cx + r + 1)
        sl = R[y0:y1, x0:x1]
        k = int(np.argmax(sl == sl.max()))  # first maximum in row-major order = smallest index
        assert (w["y"], w["x"]) == (y0 + k // sl.shape[1], x0 + k % sl.shape[1])
        assert w["rho"] == R[w["y"], w["x"]] and w["num"] == f["num_map"][w["y"], w["x"]]
        assert w["n_computed"] == sl.size


def test_paper_opta_search_pins():
    """The paper's OptA search: J's best location is J's exact argmax (the search on J is transitive
    elimination, exact for J); the answer is the localisation window's best on I around it; with J = I
    (nothing blurred) it is the exact full-search answer."""
    I = aerial_image(70, 80, 23, beta=2.2)
    m, n = 12, 10
    taps, _ = O.gauss_taps(1.5)
    J, _, _ = O.revert(I, O.blur(I, taps), m, n, O.lambda_(0.8, 0.95))
    for k in range(4):
        tpl, _ = cut_template(I, m, n, 1300 + k, 7.0)
        full = O.full_search(I, tpl)
        same = O.opta_paper_search(I, I, tpl, 3, 3, 2)
        assert (same["y"], same["x"], same["rho"]) == (full["y"], full["x"], full["rho"])
        fj = O.full_search(J, tpl)
        s = O.opta_paper_search(I, J, tpl, 3, 3, 2)
        assert s["blurred"] == (fj["y"], fj["x"], fj["rho"])
        w = O.window_search(I, tpl, fj["y"], fj["x"], 2)
        assert (s["y"], s["x"], s["rho"], s["num"]) == (w["y"], w["x"], w["rho"], w["num"])
        te = O.te_search(J, tpl, 3, 3)
        assert s["n_eliminated"] == te["n_eliminated"] and s["n_computed"] == te["n_computed"] + w["n_computed"]


# ---------------------------------------------------------------- decision maps against an independent bound

def _unit_blocks(img, m, n):
    """Every m x n block of img, mean-centred and scaled to unit length (float64 rows, row-major location
    order), and whether the block is flat (zero variance)."""
    from numpy.lib.stride_tricks import sliding_window_view
    W = sliding_window_view(img.astype(np.float64), (m, n)).reshape(-1, m * n)
    W = W - W.mean(axis=1, keepdims=True)
    nrm = np.linalg.norm(W, axis=1)
    flat = nrm < 1e-9
    U = W / np.where(flat, 1.0, nrm)[:, None]
    return U, flat


def _angle(a, b):
    """Angle between unit vectors (rows), well conditioned everywhere: 2 atan2(|a - b|, |a + b|)."""
    return 2.0 * np.arctan2(np.linalg.norm(a - b, axis=-1), np.linalg.norm(a + b, axis=-1))


def _centres(Ly, Lx, h, w):
    """Linear index of each location's group centre: groups of h x w tile the grid from (0, 0), partial last
    groups allowed, centre = origin + floor((extent - 1) / 2) (the centre rule pinned above)."""
    y, x = np.divmod(np.arange(Ly * Lx), Lx)
    gy, gx = (y // h) * h, (x // w) * w
    cy = gy + (np.minimum(h, Ly - gy) - 1) // 2
    cx = gx + (np.minimum(w, Lx - gx) - 1) // 2
    return cy * Lx + cx


BAND = 1e-7  # decisions of the float bound closer than this to the threshold are not compared


@pytest.mark.parametrize("p,q,m,n,h,w,radius,kind", [
    (40, 44, 6, 7, 3, 3, 0, "spectral"), (40, 44, 6, 7, 4, 5, 2, "spectral"),
    (36, 50, 8, 5, 5, 3, 0, "flat_patches"), (33, 41, 5, 5, 3, 4, 1, "periodic"),
    (56, 56, 16, 16, 5, 5, 0, "spectral")])
def test_te_decisions_equal_an_independent_bound(p, q, m, n, h, w, radius, kind):
    """Scan 2's decision map against the bound of Eq. 2 recomputed independently: unit blocks in float64 and
    the angle form cos|angle(t, c) - angle(c, o)|.  Every location whose independent bound lies clearly below
    the threshold must be eliminated (completeness) and every one clearly above must be matched
    (soundness); flat blocks are never eliminated."""
    img = tiny_image(p, q, 31 + p + q, kind)
    tpl, _ = cut_template(img, m, n, 7 + h, 1.0)
    te = O.te_search(img, tpl, h, w, decision=True, radius=radius)
    Ly, Lx = p - m + 1, q - n + 1
    U, flat = _unit_blocks(img, m, n)
    T, tflat = _unit_blocks(tpl, m, n)
    assert not tflat[0]
    rho = U @ T[0]
    cen = _centres(Ly, Lx, h, w)
    is_c = cen == np.arange(Ly * Lx)
    dec = te["decision"].ravel()
    assert ((dec == 1) == is_c).all()
    # the threshold: the best of the centres (and the window), an attained rho
    cand = is_c | (dec == 3)
    best0 = np.max(np.where(flat, 0.0, rho)[cand])
    assert abs(best0 - te["best0"]) <= 1e-12
    thr = te["best0"] - 1e-9
    A = _angle(T[0][None, :], U[cen])
    B = _angle(U[cen], U)
    ub = np.cos(np.abs(A - B))
    member = ~cand
    never = flat | flat[cen]
    must_go = member & ~never & (ub < thr - BAND)
    must_stay = member & (never | (ub > thr + BAND))
    assert (dec[must_go] == 0).all(), "an eliminable location was kept"
    assert (dec[must_stay] == 2).all(), "a location the bound cannot exclude was eliminated"
    assert must_go.sum() > 0 and must_stay.sum() > 0
    assert (must_go | must_stay | ~member).sum() >= Ly * Lx - 2  # the band holds (almost) nothing
    assert te["n_eliminated"] == (dec == 0).sum()


@pytest.mark.parametrize("seed,sigma,h,w,radius", [(0, 1.0, 3, 3, 2), (1, 1.5, 4, 5, 0), (2, 0.8, 5, 5, 3)])
def test_opta_decisions_equal_an_independent_bound(seed, sigma, h, w, radius):
    """The exact OptA search's decisions against the angle triangle recomputed independently: with
    A = angle(t, centre in J), B = angle(centre in J, o in J), C = angle(o in J, o in I), a location is
    eliminable iff |A - B| > C and cos(|A - B| - C) lies below the threshold (the window's best on I)."""
    I = aerial_image(44, 52, 60 + seed, beta=2.8)
    m, n = 8, 7
    taps, _ = O.gauss_taps(sigma)
    J, _, _ = O.revert(I, O.blur(I, taps), m, n, O.lambda_(0.8, 1.0))
    assert (J != I).mean() > 0.1
    tpl, _ = cut_template(I, m, n, 80 + seed, 5.0)
    s = O.opta_search(I, J, tpl, h, w, radius, decision=True)
    Ly, Lx = 44 - m + 1, 52 - n + 1
    UI, fI = _unit_blocks(I, m, n)
    UJ, fJ = _unit_blocks(J, m, n)
    T, _ = _unit_blocks(tpl, m, n)
    cen = _centres(Ly, Lx, h, w)
    dec = s["decision"].ravel()
    win = dec == 1
    best = np.max((UI @ T[0])[win & ~fI])
    assert abs(best - s["best0"]) <= 1e-12
    thr = s["best0"] - 1e-9
    A = _angle(T[0][None, :], UJ[cen])
    B = _angle(UJ[cen], UJ)
    C = _angle(UJ, UI)
    gap = np.abs(A - B) - C
    ub = np.where(gap > 0, np.cos(np.maximum(gap, 0.0)), 2.0)
    never = fI | fJ | fJ[cen]
    must_go = ~win & ~never & (gap > 1e-7) & (ub < thr - BAND)
    must_stay = ~win & (never | (gap < -1e-7) | (ub > thr + BAND))
    assert (dec[must_go] == 0).all()
    assert (dec[must_stay] == 2).all()
    assert must_go.sum() > 0 and must_stay.sum() > 0
    assert (must_go | must_stay | win).sum() >= Ly * Lx - 2


def _count_retained(U, flat, Ly, Lx, h, w, rho_th, C=None, fI=None, estimate=0, rho_tc=0.0):
    """Retained-location count of EGS recomputed from unit blocks (the reading of each estimate stated in
    the oracle).  Returns (count, locations within the band of the threshold)."""
    cen = _centres(Ly, Lx, h, w)
    is_c = cen == np.arange(Ly * Lx)
    B = _angle(U[cen], U)
    never = flat | flat[cen]
    if C is not None:
        never = never | fI
    if estimate == 0:
        thr = math.sqrt(1.0 - rho_th * rho_th)
        val = np.cos(B + (C if C is not None else 0.0))
        kept, near = val < thr, np.abs(val - thr) < BAND
    else:
        A = math.acos(rho_tc)
        gap = np.abs(A - B) - (C if C is not None else 0.0)
        val = np.where(gap > 0, np.cos(np.maximum(gap, 0.0)), 2.0)
        kept, near = val > rho_th, (np.abs(val - rho_th) < BAND) | (np.abs(gap) < 1e-7)
    counted = np.ones(Ly * Lx, bool) if C is not None else ~is_c
    kept = counted & (never | kept)
    near = counted & ~never & near
    return int(kept.sum()), int(near.sum())


@pytest.mark.parametrize("estimate,rho_tc", [(0, 0.0), (1, 0.0), (1, 0.35), (1, -0.2)])
def test_egs_counts_equal_an_independent_count(estimate, rho_tc):
    """EGS's retained counts, without blur (Prop. 3.2, Eq. 15) and with the angle to the original added
    (the exact OptA search's count), and Prop. 3.1's two-root estimate at an assumed rho_tc, against counts
    recomputed from unit blocks."""
    I = aerial_image(48, 56, 91, beta=2.8)
    m, n = 8, 8
    taps, _ = O.gauss_taps(1.0)
    J, _, _ = O.revert(I, O.blur(I, taps), m, n, O.lambda_(0.8, 1.0))
    assert (J != I).mean() > 0.1
    Ly, Lx = 48 - m + 1, 56 - n + 1
    UJ, fJ = _unit_blocks(J, m, n)
    UI, fI = _unit_blocks(I, m, n)
    for use_c in (False, True):
        c = O.blurcorr(I, J, m, n) if use_c else None
        e = O.egs(J, m, n, c=c, estimate=estimate, rho_tc=rho_tc)
        assert e["trace"]
        for step in e["trace"]:
            want, near = _count_retained(UJ, fJ, Ly, Lx, step["h"], step["w"], 0.8,
                                         C=_angle(UJ, UI) if use_c else None, fI=fI, estimate=estimate,
                                         rho_tc=rho_tc)
            assert want - near <= step["cr"] <= want + near
            assert near <= 2


def test_egs_two_dimensional_ascent():
    """shape 1 evaluates (h+dh, w), (h, w+dw), (h+dh, w+dw) from the last accepted size and accepts the
    cheapest when it lowers the cost by more than xi; each candidate's cost is mn (groups + retained)."""
    img = aerial_image(72, 80, 5, beta=2.6)
    m = n = 10
    Ly, Lx = 72 - m + 1, 80 - n + 1
    U, flat = _unit_blocks(img, m, n)
    e = O.egs(img, m, n, shape=1)
    tr = e["trace"]
    prev, cur, i = m * n * Ly * Lx, None, 0
    while i < len(tr):
        if cur is None:
            cands = [(3, 3)]
        else:
            cands = [(cur[0] + 2, cur[1]), (cur[0], cur[1] + 2), (cur[0] + 2, cur[1] + 2)]
        cands = [c for c in cands if c[0] <= min(33, Ly) and c[1] <= min(33, Lx)]
        rows = tr[i:i + len(cands)]
        assert [(r["h"], r["w"]) for r in rows] == cands
        for r in rows:
            gy, gx = -(-Ly // r["h"]), -(-Lx // r["w"])
            assert r["cc"] == gy * gx
            want, near = _count_retained(U, flat, Ly, Lx, r["h"], r["w"], 0.8)
            assert want - near <= r["cr"] <= want + near
            assert r["ct"] == m * n * (r["cc"] + r["cr"])
        i += len(cands)
        best = min(range(len(rows)), key=lambda k: (rows[k]["ct"], k))
        ok = (prev - rows[best]["ct"]) > 0.005 * prev
        assert [r["accepted"] for r in rows] == [ok and k == best for k in range(len(rows))]
        if not ok:
            break
        prev, cur = rows[best]["ct"], (rows[best]["h"], rows[best]["w"])
    assert i == len(tr)
    assert (e["h"], e["w"]) == (cur if cur else (1, 1)) and e["cost"] == prev
    assert any(r["h"] != r["w"] for r in tr)


def test_paper_conditioning_is_alg3_as_printed():
    """paper=True: every accepted iterate's EGS is EGS on the blurred image alone (no angle to the original),
    warm-started at the previous size; the final image keeps every blur correlation >= lambda; the paper's
    conditioning differs from the exact one's on an input where blur is accepted."""
    I = aerial_image(96, 96, 7002, beta=2.6)
    m = n = 24
    kw = dict(rho_max=1.0, nthreads=4)
    op = O.opta(I, m, n, paper=True, **kw)
    acc = [s for s in op["trace"] if s["accepted"]]
    assert len(acc) >= 3 and len({s["h"] for s in acc}) >= 2
    J = op["image"]
    num, dj, di = O.blurcorr(I, J, m, n)
    lam = O.lambda_(0.8, 1.0)
    for l in range(len(num)):
        assert dj[l] != 0 and di[l] != 0 and O.rho(num[l], dj[l], di[l]) >= lam
    prev_h = acc[-2]["h"]
    e = O.egs(J, m, n, h0=prev_h, w0=prev_h)
    assert (e["h"], e["w"], e["cost"]) == (op["h"], op["w"], op["cost"])
    ex = O.opta(I, m, n, paper=False, **kw)
    assert ex["trace"] != op["trace"]


def test_detection_floor_semantics():
    """With a floor the threshold is max(best0, floor): at or below the true maximum the answer is the
    full search's and nothing eliminated reaches the floor; above it every eliminated location lies below the
    floor (the full map says so), and elimination only grows with the floor."""
    img = aerial_image(64, 72, 77, beta=2.2)
    m, n = 10, 9
    for k in range(3):
        tpl, _ = cut_template(img, m, n, 300 + k, 12.0, affine=True)
        full = O.full_search(img, tpl, maps=True)
        rho = full["rho_map"].ravel()
        base = O.te_search(img, tpl, 3, 3, decision=True)
        prev = base["n_eliminated"]
        for fl in sorted((full["rho"] - 0.05, full["rho"], full["rho"] + 1e-6, 0.95, 0.999)):
            s = O.te_search(img, tpl, 3, 3, decision=True, floor=fl)
            dec = s["decision"].ravel()
            assert (rho[dec == 0] < max(fl, s["best0"])).all()
            assert s["n_eliminated"] >= prev
            prev = s["n_eliminated"]
            if fl <= full["rho"]:
                assert (s["y"], s["x"], s["rho"]) == (full["y"], full["x"], full["rho"])
            assert s["rho"] <= full["rho"]
        J = O.blur(img, O.gauss_taps(0.8)[0])
        J, _, _ = O.revert(img, J, m, n, O.lambda_(0.8, 1.0))
        for fl in (full["rho"] - 0.1, 0.999):
            s = O.opta_search(img, J, tpl, 3, 3, 2, decision=True, floor=fl)
            dec = s["decision"].ravel()
            assert (rho[dec == 0] < max(fl, s["best0"])).all()
            if fl <= full["rho"]:
                assert (s["y"], s["x"], s["rho"]) == (full["y"], full["x"], full["rho"])
