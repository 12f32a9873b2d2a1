"""zts_search_device_noalloc: the allocation-free variant of zts_search_device (collected last).

Its query scratch lives in the library's static device array.  Each call is
compared field by field with zts_search_device on the same inputs (and the
exact modes with the oracle's answer), on consecutive calls whose second input
is smaller than the first, so a stale part of the shared array would show.
"""

import numpy as np
import pytest

import oracle as O
from synth import aerial_image, cut_template

pytestmark = pytest.mark.gpu

Z = pytest.importorskip("paper_1407_3535_amd")

FIELDS = ("y", "x", "rho", "rho32", "num", "den_t", "den_r", "n_locations", "n_centres", "n_eliminated",
          "n_survivors", "n_computed", "group_h", "group_w", "best0", "best0_y", "best0_x", "above_floor")
E_SIZE, E_ARG, E_NOTPREPARED = -2, -1, -12


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs():
    big = aerial_image(300, 280, 4242, beta=2.0)
    small = aerial_image(120, 110, 4243, beta=2.2)
    tb, _ = cut_template(big, 24, 24, 4244, 6.0)
    ts, _ = cut_template(small, 12, 13, 4245, 6.0)
    return (big, tb), (small, ts)


MODES = [("full", {}), ("te_fixed", dict(group_h=3, group_w=4)), ("egs", {}), ("egs", dict(refine_radius=2)),
         ("opta", {}), ("opta", dict(refine_radius=3)), ("opta_paper", {})]


@pytest.mark.parametrize("mode,kw", MODES, ids=[f"{m}{'-' + str(k) if k else ''}" for m, k in MODES])
def test_noalloc_equals_search_device_twice(torch_gpu, mode, kw):
    torch = torch_gpu
    pairs = _inputs()
    with Z.Searcher(0) as S:
        ids = [S.load(img) for img, _ in pairs]
        for i, (img, tpl) in zip(ids, pairs):
            S.prepare(i, tpl.shape[0], tpl.shape[1], mode, **kw)
        params = Z.zts_params_default(**kw)
        for rep in range(2):
            for i, (img, tpl) in zip(ids, pairs):  # the second input is the smaller one
                print(f"noalloc {mode} {kw} rep {rep} img {img.shape} tpl {tpl.shape}", flush=True)
                t = torch.from_numpy(tpl).cuda()
                want = Z.zts_search_device(S.ctx, i, t, mode, params)
                got = Z.zts_search_device_noalloc(S.ctx, i, t, mode, params)
                torch.cuda.synchronize()
                for k in FIELDS:
                    assert got[k] == want[k], f"{mode} {img.shape}: {k} noalloc={got[k]} device={want[k]}"
                if mode != "opta_paper":
                    ref = O.full_search(img, tpl)
                    for k in ("y", "x", "rho", "num", "den_t", "den_r"):
                        assert got[k] == ref[k], f"{mode}: {k} against the oracle"
                    assert abs(got["rho32"] - ref["rho"]) <= 1e-6


def test_noalloc_two_contexts_alternate(torch_gpu):
    torch = torch_gpu
    (big, tb), (small, ts) = _inputs()
    with Z.Searcher(0) as A, Z.Searcher(0) as B:
        ia, ib = A.load(big), B.load(small)
        A.prepare(ia, *tb.shape, "egs")
        B.prepare(ib, *ts.shape, "opta")
        ta, tsm = torch.from_numpy(tb).cuda(), torch.from_numpy(ts).cuda()
        for _ in range(3):
            ga = Z.zts_search_device_noalloc(A.ctx, ia, ta, "egs")
            gb = Z.zts_search_device_noalloc(B.ctx, ib, tsm, "opta")
            wa = Z.zts_search_device(A.ctx, ia, ta, "egs")
            wb = Z.zts_search_device(B.ctx, ib, tsm, "opta")
            for k in FIELDS:
                assert ga[k] == wa[k] and gb[k] == wb[k], k


def test_noalloc_refusals(torch_gpu):
    torch = torch_gpu
    (big, tb), _ = _inputs()
    with Z.Searcher(0) as S:
        i = S.load(big)
        t = torch.from_numpy(tb).cuda()
        # nothing resident for this size yet: no statistics, no tables
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "full")
        assert e.value.code == E_NOTPREPARED
        S.prepare(i, *tb.shape, "full")
        Z.zts_search_device_noalloc(S.ctx, i, t, "full")
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "egs")
        assert e.value.code == E_NOTPREPARED
        S.prepare(i, *tb.shape, "egs")
        Z.zts_search_device_noalloc(S.ctx, i, t, "egs")
        # tables prepared with other parameters do not serve
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "egs", Z.zts_params_default(rho_th=0.9))
        assert e.value.code == E_NOTPREPARED
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "full_mfma")
        assert e.value.code == E_ARG
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "egs", Z.zts_params_default(margin=-1.0))
        assert e.value.code == E_ARG


def test_noalloc_scratch_limit(torch_gpu):
    """A query whose scratch exceeds the 96 MiB array is refused before anything is launched; the next call
    on the same GPU still gives the right answer."""
    torch = torch_gpu
    rng = np.random.default_rng(99)
    img = rng.integers(0, 256, (6000, 6000), dtype=np.uint8)  # 1 x 2 groups: 1.79e7 groups, 8 B each
    tpl = img[1000:1016, 2000:2016].copy()
    (big, tb), _ = _inputs()
    with Z.Searcher(0) as S:
        i = S.load(img)
        S.prepare(i, 16, 16, "te_fixed", group_h=1, group_w=2)
        t = torch.from_numpy(tpl).cuda()
        p = Z.zts_params_default(group_h=1, group_w=2)
        with pytest.raises(Z.ZtsError) as e:
            Z.zts_search_device_noalloc(S.ctx, i, t, "te_fixed", p)
        assert e.value.code == E_SIZE
        g = Z.zts_search_device(S.ctx, i, t, "te_fixed", p)
        assert (g["y"], g["x"]) == (1000, 2000)
        S.unload(i)
        j = S.load(big)
        S.prepare(j, *tb.shape, "te_fixed", group_h=1, group_w=2)
        tt = torch.from_numpy(tb).cuda()
        got = Z.zts_search_device_noalloc(S.ctx, j, tt, "te_fixed", p)
        want = Z.zts_search_device(S.ctx, j, tt, "te_fixed", p)
        for k in FIELDS:
            assert got[k] == want[k], k
