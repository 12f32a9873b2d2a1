"""GPU tests of the batch autotuner (zts_tune_batch): measured routes, the
crossover rule, answers unchanged under any route, and the tune_cache file."""

import numpy as np
import pytest

import oracle as O
from synth import aerial_image, cut_template

pytestmark = pytest.mark.gpu

Z = pytest.importorskip("paper_1407_3535_amd")

KEYS = ("y", "x", "rho", "num", "den_t", "den_r")
INT32_MAX = 2 ** 31 - 1


def gpu_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def crossover(single, shared):
    if not single > 0.0:
        return 1
    for T in range(2, 17):
        if shared < T * single:
            return T
    return INT32_MAX


def test_tune_routes_answers_and_cache(tmp_path):
    gpu_or_skip()
    img = aerial_image(200, 240, 101)
    cache = tmp_path / "tune.txt"
    sizes = [(16, 16), (24, 40), (48, 48)]
    with Z.Searcher(0, tune_cache=str(cache)) as S:
        i = S.load(img)
        ents = S.tune_batch(i, sizes)
        for (m, n), e in zip(sizes, ents):
            print(e, flush=True)
            assert (e["m"], e["n"]) == (m, n)
            assert e["single_ms"] > 0.0 and e["shared_ms"] > 0.0
            assert e["multi_min"] == crossover(e["single_ms"], e["shared_ms"])
        # groups on both sides of each crossover give the oracle's answers
        for k, (m, n) in enumerate(sizes):
            for T in (1, 3, 6):
                tpls = [cut_template(img, m, n, 900 + 10 * k + j, 4.0)[0] for j in range(T)]
                res = S.search_batch(i, tpls)
                for t, r in zip(tpls, res):
                    o = O.full_search(img, t)
                    for key in KEYS:
                        assert r[key] == o[key], (m, n, T, key)
        with pytest.raises(Z.ZtsError) as e:
            S.tune_batch(i, [(8, 200)])
        assert e.value.code == -2
    lines = [l.split() for l in cache.read_text().splitlines() if l.strip()]
    assert sorted((int(l[1]), int(l[2])) for l in lines) == sorted(sizes)
    assert len({l[0] for l in lines}) == 1
    # a new context reads the file; its batches still give the same answers
    with Z.Searcher(0, tune_cache=str(cache)) as S2:
        i = S2.load(img)
        tpls = [cut_template(img, 24, 40, 950 + j, 4.0)[0] for j in range(4)]
        for t, r in zip(tpls, S2.search_batch(i, tpls)):
            o = O.full_search(img, t)
            assert (r["y"], r["x"], r["rho"]) == (o["y"], o["x"], o["rho"])
