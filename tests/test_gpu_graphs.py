"""GPU tests of replayed query graphs.

A query whose launch arguments were seen before in the same slot is captured
into a HIP graph on its second occurrence and replayed after that (the
template bytes live in the slot's buffer, so a replay searches whatever
template was staged); with timing=1 the same query runs kernel by kernel with
an event after each.  Every replay, with eager work and synchronisations in
between, must give the oracle's answer and the oracle's method counts, exactly
as the eager runs do."""

import numpy as np
import pytest

import oracle as O
from synth import aerial_image, cut_template

pytestmark = pytest.mark.gpu

Z = pytest.importorskip("paper_1407_3535_amd")

RHO32_TOL = 1e-6
KEYS = ("y", "x", "rho", "num", "den_t", "den_r")
COUNTS = ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed", "group_h", "group_w")


def gpu_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_graph_replays_match_oracle():
    gpu_or_skip()
    img = aerial_image(220, 260, 91)
    with Z.Searcher(0) as S:
        i = S.load(img)
        info = S.prepare(i, 20, 20, "egs")
        h, w = info["h"], info["w"]
        oo = O.opta(img, 16, 16, max_iters=3)
        S.prepare(i, 16, 16, "opta", max_iters=3)
        cases = [("egs", 20, 20, {}, lambda t: O.te_search(img, t, h, w)),
                 ("egs", 20, 20, {"refine_radius": 2}, lambda t: O.te_search(img, t, h, w, radius=2)),
                 ("te_fixed", 17, 31, {"group_h": 3, "group_w": 5},
                  lambda t: O.te_search(img, t, 3, 5)),
                 ("opta", 16, 16, {"max_iters": 3},
                  lambda t: O.opta_search(img, oo["image"], t, oo["h"], oo["w"], oo["radius"])),
                 ("full", 12, 18, {}, None)]
        for rep in range(5):
            for k, (mode, m, n, kw, method) in enumerate(cases):
                t, _ = cut_template(img, m, n, 300 + 17 * rep + k, 5.0)
                print(f"rep {rep} case {k} {mode} {m}x{n}", flush=True)
                g = S.search(i, t, mode, **kw)
                full = O.full_search(img, t)
                for key in KEYS:
                    assert g[key] == full[key], (rep, k, key)
                assert abs(g["rho32"] - full["rho"]) <= RHO32_TOL
                if method is not None:
                    o = method(t)
                    for key in COUNTS:
                        assert g[key] == o[key], (rep, k, key, g[key], o[key])
                    assert g["best0"] == o["best0"], (rep, k)
                assert g["device_ms"] > 0.0 and g["phase_ms"] == [0.0] * 6
                # the same query launched kernel by kernel with its events
                gt = S.search(i, t, mode, timing=1, **kw)
                for key in KEYS + COUNTS:
                    assert gt[key] == g[key], (rep, k, key)
                assert gt["phase_ms"][0] > 0.0, gt["phase_ms"]
                if mode != "full":
                    assert gt["phase_ms"][2] > 0.0 and gt["phase_ms"][3] > 0.0, gt["phase_ms"]
                # eager work between replays: a decision-map query (never
                # captured) and a batched launch
                if k == 1:
                    gd, dec = S.search(i, t, "te_fixed", decision=True, group_h=2, group_w=2)
                    assert (gd["y"], gd["x"]) == (full["y"], full["x"])
                    assert dec.shape == (img.shape[0] - m + 1, img.shape[1] - n + 1)
                if k == 3:
                    rb = S.search_batch(i, [t, t])
                    assert (rb[0]["y"], rb[0]["x"]) == (full["y"], full["x"])


def test_batch_graph_replays_match_oracle():
    """A repeated batch plan (same sizes and buffers) replays its captured
    kernels; new template contents are staged each call."""
    gpu_or_skip()
    img = aerial_image(180, 210, 93)
    with Z.Searcher(0) as S:
        i = S.load(img)
        shapes = [(16, 16), (16, 16), (16, 16), (20, 36), (33, 17)]
        for rep in range(4):
            tpls = [cut_template(img, m, n, 700 + 13 * rep + k, 5.0)[0] for k, (m, n) in enumerate(shapes)]
            print(f"batch rep {rep}", flush=True)
            res = S.search_batch(i, tpls)
            for t, r in zip(tpls, res):
                o = O.full_search(img, t)
                for key in KEYS:
                    assert r[key] == o[key], (rep, t.shape, key)
            S.search(i, tpls[0], "full")  # eager work between the replays
