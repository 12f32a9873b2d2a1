"""GPU parity at full size: every workload against the oracle's answers on the same inputs.

The answers were computed once by the CPU oracle (tests/golden/make_full_size.py, which calls only oracle/
and synth/) and are stored in tests/golden/full_size.json keyed by the SHA-256 of the input bytes; each test
regenerates the inputs, checks their hashes, and compares element by element: the location, the exact
integers N, D_t, D_r and the binary64 rho (bit for bit), binary32 rho within 1e-6, and where stored the
preparation traces, the conditioned image's hash and the counts.
"""

import hashlib
import json
import os

import numpy as np
import pytest

from synth import serving_queries, workload

pytestmark = pytest.mark.gpu

Z = pytest.importorskip("paper_1407_3535_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")
ANSWER = ("y", "x", "rho", "num", "den_t", "den_r")
COUNTS = ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed", "best0")
TRACE = ("k", "d", "passes", "reverted", "h", "w", "cost", "accepted")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = Z.Searcher(0)
    yield s
    s.close()


def same(g, o, keys, what):
    for k in keys:
        assert g[k] == o[k], f"{what}: {k} gpu={g[k]} oracle={o[k]}"
    if "rho" in keys:
        assert abs(g["rho32"] - o["rho"]) <= 1e-6, what


def same_conditioning(info, J, want, what):
    assert (info["h"], info["w"], info["radius"], info["cost"]) == (want["h"], want["w"], want["radius"],
                                                                      want["cost"]), what
    got = [{k: s[k] for k in TRACE} for s in info["opta"]]
    exp = [{k: (bool(s[k]) if k == "accepted" else s[k]) for k in TRACE} for s in want["trace"]]
    assert got == exp, what
    assert sha(J) == want["image_sha256"], what


def test_workload2_against_oracle(S, golden):
    """2048x2048, one 64x64 template: plain answer in every mode; Alg. 2's trace and the two-scan counts;
    both forms of Alg. 3's conditioning (trace, conditioned image) and the counts of the searches."""
    e = golden["2"]
    w = workload(2)
    img = w["images"][0]
    tpl, loc, _ = w["templates"][0]
    assert sha(img) == e["image_sha256"] and sha(tpl) == e["template_sha256"]
    m, n = tpl.shape
    i = S.load(img)
    for mode in ("full", "full_mfma"):
        same(S.search(i, tpl, mode), e["plain"], ANSWER, mode)
    info = S.prepare(i, m, n, "egs")
    assert (info["h"], info["w"], info["cost"]) == (e["egs"]["h"], e["egs"]["w"], e["egs"]["cost"])
    assert info["egs"] == [{**s, "accepted": bool(s["accepted"])} for s in e["egs"]["trace"]]
    for radius in (0, 2):
        g = S.search(i, tpl, "egs", refine_radius=radius)
        same(g, e["plain"], ANSWER, f"egs r{radius}")
        same(g, e["egs"][f"search_radius{radius}"], COUNTS, f"egs r{radius} counts")
    info = S.prepare(i, m, n, "opta")
    same_conditioning(info, S.prep_image(i, m, n, "opta"), e["opta"], "opta conditioning")
    g = S.search(i, tpl, "opta", refine_radius=e["opta"]["search_radius"])
    same(g, e["plain"], ANSWER, "opta")
    same(g, e["opta"]["search"], COUNTS, "opta counts")
    info = S.prepare(i, m, n, "opta_paper")
    same_conditioning(info, S.prep_image(i, m, n, "opta_paper"), e["opta_paper"], "paper conditioning")
    g = S.search(i, tpl, "opta_paper")
    same(g, e["opta_paper"]["search"], ANSWER + ("n_locations", "n_centres", "n_eliminated", "n_survivors",
                                                  "n_computed"), "paper search")
    S.unload(i)


def test_workload3_against_oracle(S, golden):
    """8192x8192 with clouds, 8 templates of 32, 64 and 128 px (affine change and noise): the exact OptA
    search's answer equals the oracle's plain answer for every template, its counts equal the oracle's
    OptA search, and the conditioning of each size equals the oracle's; the plain and int8-MFMA searches
    give the same answers."""
    e = golden["3"]
    w = workload(3)
    img = w["images"][0]
    assert sha(img) == e["image_sha256"]
    i = S.load(img)
    for size, want in e["opta"].items():
        m = int(size)
        print(f"workload 3: conditioning {m}x{m}", flush=True)
        info = S.prepare(i, m, m, "opta")
        same_conditioning(info, S.prep_image(i, m, m, "opta"), want, f"conditioning {m}")
    assert len(e["templates"]) == len(w["templates"])
    for k, ((tpl, loc, _), rec) in enumerate(zip(w["templates"], e["templates"])):
        assert sha(tpl) == rec["template_sha256"]
        print(f"workload 3: template {k} {tpl.shape}", flush=True)
        g = S.search(i, tpl, "opta", refine_radius=2)
        assert rec["opta_search_radius"] == max(e["opta"][str(tpl.shape[0])]["radius"], 2)
        same(g, rec["plain"], ANSWER, f"template {k} opta")
        same(g, rec["opta_search"], COUNTS, f"template {k} opta counts")
        for mode in ("full_mfma", "egs"):
            same(S.search(i, tpl, mode), rec["plain"], ANSWER, f"template {k} {mode}")
    S.unload(i)


def test_workload4_against_oracle(S, golden):
    """4096x4096, 64 templates of sizes 16..128 in one batched int8-MFMA call: every answer equals the
    oracle's plain answer."""
    e = golden.get("4")
    w = workload(4)
    if e is None or len(e["templates"]) < len(w["templates"]):
        pytest.skip("the oracle's answers for this workload are not complete in tests/golden/full_size.json")
    img = w["images"][0]
    assert sha(img) == e["image_sha256"]
    tpls = [t for t, _, _ in w["templates"]]
    for t, rec in zip(tpls, e["templates"]):
        assert sha(t) == rec["template_sha256"]
    i = S.load(img)
    res = S.search_batch(i, tpls)
    for k, (r, rec) in enumerate(zip(res, e["templates"])):
        assert r["status"] == 0
        same(r, rec["plain"], ANSWER, f"batch template {k} {tpls[k].shape}")
    S.unload(i)


def test_workload5_against_oracle(S, golden):
    """The serving workload's first 64 queries (4 resident images, half of the queries noise patches with no
    true match), served concurrently in three modes (fused int8-MFMA batches, EGS and exact OptA with
    refinement): every served answer equals the oracle's plain answer."""
    e = golden.get("5")
    if e is None or len(e["templates"]) < e.get("queries", 64):
        pytest.skip("the oracle's answers for this workload are not complete in tests/golden/full_size.json")
    imgs = workload(5)["images"]
    assert [sha(im) for im in imgs] == e["image_sha256"]
    qs = serving_queries(imgs, e["queries"])
    with Z.Searcher(0, max_inflight=4) as T:
        ids = [T.load(im) for im in imgs]
        modes = [("full_mfma", {}), ("egs", {}), ("opta", dict(refine_radius=2))]
        tickets = []
        for k, ((t, j, _), rec) in enumerate(zip(qs, e["templates"])):
            assert sha(t) == rec["template_sha256"] and j == rec["image"]
            mode, kw = modes[k % 3]
            tickets.append((k, mode, T.submit(ids[j], t, mode, **kw)))
        for k, mode, tk in tickets:
            st, r = T.wait(tk)
            assert st == 0, (k, mode, st)
            same(r, e["templates"][k]["plain"], ANSWER, f"served query {k} ({mode})")
