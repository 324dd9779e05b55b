"""The C-ABI library loads, exports every entry point its header declares and
rejects bad plans on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2506_22935_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "graf_af.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libgraf_af.so not built")
    return L.lib()


def test_header_declares_the_bound_names():
    assert set(declared()) == set(L.SIGNATURES)


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in L.STATUS:
        assert lib.af_status_string(code)
    assert lib.af_version() >= 100


def _create(lib, waves, **opt):
    arr = (L.AfWave * len(waves))()
    off = 0
    goff = 0
    for i, (n, m, T) in enumerate(waves):
        arr[i].n, arr[i].m, arr[i].max_lag = n, m, T
        arr[i].h_tau, arr[i].h_k, arr[i].flags = 1, 1, 0
        arr[i].s_off, arr[i].grid_off = off, goff
        off += n
        goff += (2 * (n - 1 if T < 0 else T) + 1) * m
    for k, v in opt.get("fields", {}).items():
        setattr(arr[0], k, v)
    opts = L.AfPlanOpts(eps=1e-12, store_mode=opt.get("store_mode", 0), budget_bytes=0, variant=-1,
                        segment_iters=0, launch_mode=opt.get("launch_mode", 0))
    h = ctypes.c_void_p()
    rc = lib.af_plan_create(len(waves), arr, ctypes.byref(opts), ctypes.byref(h))
    if rc == 0:
        lib.af_plan_destroy(h)
    return rc


@pytest.mark.parametrize("waves,code", [
    ([(100, 128, -1)], -2),     # M < 2N
    ([(64, 100, -1)], -2),      # M not a power of two
    ([(32, 64, -1)], -2),       # M below the smallest supported size
    ([(64, 65536, -1)], -2),    # M above the largest supported size
    ([(64, 128, 64)], -1),      # lag window beyond N - 1
    ([(0, 128, -1)], -1),       # empty waveform
    ([(64, 128, -2)], -1),      # bad lag window
])
def test_plan_validation(lib, waves, code):
    assert _create(lib, waves) == code


def test_plan_validation_fields(lib):
    assert _create(lib, [(64, 128, -1)], fields={"flags": 2}) == -1
    # periodic AF: m = n, a power of two in [64, 4096], every lag, h <= n/2
    per = {"flags": L.AF_WAVE_PERIODIC}
    assert _create(lib, [(64, 128, -1)], fields=per) == -1
    assert _create(lib, [(64, 64, 10)], fields=per) == -1
    assert _create(lib, [(64, 64, -1)], fields=dict(per, h_tau=33)) == -1
    assert _create(lib, [(96, 96, -1)], fields=per) == -2
    assert _create(lib, [(32, 32, -1)], fields=per) == -2
    assert _create(lib, [(8192, 8192, -1)], fields=per) == -2
    assert _create(lib, [(64, 64, -1)], fields=per) not in (-1, -2)
    assert _create(lib, [(4096, 4096, -1)], fields=per) not in (-1, -2)
    assert _create(lib, [(64, 128, -1)], fields={"grid_off": 2}) == -1
    assert _create(lib, [(64, 128, -1)], fields={"h_tau": -1}) == -1
    assert _create(lib, [(64, 128, -1)], store_mode=3) == -1
    assert _create(lib, [(64, 128, -1)], launch_mode=2) == -1
    assert _create(lib, [(64, 128, -1)], launch_mode=-1) == -1


def test_null_arguments(lib):
    assert lib.af_plan_create(1, None, None, None) == -1
    assert lib.af_forward(None, None, None, None, None, None, 0, None) == -1
    assert lib.af_backward(None, None, None, None, None, 0, None) == -1
    assert lib.af_phase_to_signal(None, None, 5, None) == -1
    sz = ctypes.c_size_t()
    assert lib.af_plan_workspace_size(None, ctypes.byref(sz)) == -1
    # the composite-loss, projection, scenario and cross-AF entry points check
    # their arguments on the host before any device work
    assert lib.af_project(None, None, None, 0, None, None) == -1
    assert lib.af_scenario_combine(None, 2, None, None, None, None) == -1
    assert lib.af_cross_workspace_size(None, ctypes.byref(sz)) == -1
    assert lib.af_cross_forward(None, None, None, None, None, None, None) == -1
    assert lib.af_cross_backward(None, None, None, None, None, None, None, 0, None) == -1
    assert lib.af_spectral_variance(None, None, None, None, None, 0, None) == -1


def test_gemm_config_resolution(lib):
    # automatic tiles and splits (the host rule without a device assumes 256
    # compute units): a tile that divides the shape, a split that divides k
    # into whole k tiles, workspace for the partial sums exactly when split
    from paper_2506_22935_amd import mlp as M
    bk = {1: 64, 2: 64, 3: 64, 4: 64, 5: 128, 6: 128, 7: 128, 8: 128}
    bm = {1: 128, 2: 128, 3: 64, 4: 64, 5: 128, 6: 128, 7: 64, 8: 64}
    bn = {1: 128, 2: 64, 3: 128, 4: 64, 5: 128, 6: 64, 7: 128, 8: 64}
    for m, n, k in [(4096, 1024, 1024), (4096, 1024, 64), (4096, 256, 1024), (1024, 1024, 4096), (256, 1024, 4096),
                    (1024, 64, 4096), (128, 64, 192), (64, 64, 64)]:
        t, s, b = M.gemm_config(m, n, k)
        assert m % bm[t] == 0 and n % bn[t] == 0 and k % (bk[t] * s) == 0, (m, n, k, t, s)
        assert b == (s * m * n * 4 if s > 1 else 0)
    assert M.gemm_config(1024, 1024, 4096)[1] > 1               # few output tiles: k is split
    assert M.gemm_config(4096, 1024, 1024)[1] == 1              # enough output tiles: no split
    assert M.gemm_config(256, 384, 768, tile=3, split_k=12) == (3, 12, 12 * 256 * 384 * 4)
    for bad in [(100, 64, 64, 0, 0), (128, 64, 96, 0, 0), (64, 64, 64, 1, 0), (128, 128, 128, 5, 2),
                (128, 128, 1024, 0, 17), (128, 128, 128, 9, 0)]:
        with pytest.raises(L.AfError):
            M.gemm_config(*bad)
    n = ctypes.c_size_t()
    assert lib.af_colsum_workspace_size(4096, 1024, ctypes.byref(n)) == 0 and n.value % (1024 * 4) == 0
