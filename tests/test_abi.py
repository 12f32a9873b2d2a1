"""The C-ABI library loads and exports what include/zts.h declares (CPU only)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zts.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(zts_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    Z = pytest.importorskip("paper_1407_3535_amd")
    assert sorted(Z.EXPORTS) == declared()


def test_library_exports_every_declared_symbol():
    Z = pytest.importorskip("paper_1407_3535_amd")
    L = Z.lib()
    for name in declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", Z.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (zts_\w+)", out))
    assert set(declared()) <= exported


def test_struct_layouts_match_the_header(tmp_path):
    Z = pytest.importorskip("paper_1407_3535_amd")
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include "%s"\nint main(void){printf("%%zu %%zu %%zu %%zu %%zu %%zu %%zu\\n",'
                    'sizeof(zts_result), sizeof(zts_prep_info), sizeof(zts_params), sizeof(zts_ctx_params),'
                    'sizeof(zts_egs_step), sizeof(zts_opta_step), sizeof(zts_tune_entry));return 0;}\n' % HEADER)
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", str(prog), "-o", str(exe)])
    sizes = list(map(int, subprocess.check_output([str(exe)]).split()))
    assert sizes == [ctypes.sizeof(Z.Result), ctypes.sizeof(Z.PrepInfo), ctypes.sizeof(Z.Params),
                     ctypes.sizeof(Z.CtxParams), ctypes.sizeof(Z.EgsStep), ctypes.sizeof(Z.OptaStep),
                     ctypes.sizeof(Z.TuneEntry)]


def test_defaults_are_the_papers():
    Z = pytest.importorskip("paper_1407_3535_amd")
    p = Z.zts_params_default()
    assert (p.rho_th, p.rho_max, p.xi) == (0.80, 0.95, 0.005)
    assert (p.group_h, p.group_w) == (5, 5)
    assert Z.zts_status_str(-3) == "template has zero variance"


def test_no_device_is_a_clean_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    Z = pytest.importorskip("paper_1407_3535_amd")
    with pytest.raises(Z.ZtsError) as e:
        Z.zts_create(0)
    assert e.value.code == -10


def test_params_check_rejects_out_of_range_values():
    """Every entry point that takes parameters applies zts_params_check first; this exercises it on the host
    (no device): a negative or NaN margin could eliminate the true maximum, a huge refinement radius would
    overflow the window's record count."""
    Z = pytest.importorskip("paper_1407_3535_amd")
    assert Z.zts_params_check(Z.zts_params_default()) == 0
    nan, inf = float("nan"), float("inf")
    bad = [dict(margin=-1e-9), dict(margin=nan), dict(margin=inf), dict(refine_radius=-1),
           dict(refine_radius=256), dict(refine_radius=23170), dict(sigma_step=0.0), dict(sigma_step=nan),
           dict(xi=-0.01), dict(xi=nan), dict(rho_th=1.0), dict(rho_th=-1.0), dict(rho_th=nan),
           dict(rho_max=1.0001), dict(accept_xi=1.0), dict(accept_xi=-1.0), dict(dh=0, dw=0), dict(dh=-1),
           dict(h0=0), dict(group_h=0), dict(h_max=0), dict(blur_kind=2), dict(max_iters=16), dict(max_iters=-1),
           dict(egs_estimate=2), dict(egs_shape=-1), dict(rho_tc=1.0), dict(rho_floor=nan), dict(floor_prune=2)]
    for kw in bad:
        assert Z.zts_params_check(Z.zts_params_default(**kw)) == -1, kw
    good = [dict(margin=0.0), dict(refine_radius=255), dict(rho_max=1.0), dict(accept_xi=-0.5),
            dict(egs_estimate=1, rho_tc=0.3), dict(egs_shape=1), dict(rho_floor=0.7, floor_prune=1),
            dict(blur_kind=0, sigma_step=0.0)]
    for kw in good:
        assert Z.zts_params_check(Z.zts_params_default(**kw)) == 0, kw
