"""C-ABI checks that need no GPU: the library loads, exports every function
include/cvib.h declares, the header's struct layouts match the binding, and
argument validation fails with CV_EINVAL before touching a device."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cvib.h")


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    if not os.path.exists(cv.LIB_PATH):
        from paper_2507_22901_amd import _build
        _build.build()
    cv.lib()
    return cv


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(cv_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(cv):
    names = declared_functions()
    assert len(names) >= 8
    L = cv.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(cv.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", cv.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = sorted(set(re.findall(r" T (cv_\w+)", out)))
    assert exported == names


def test_struct_layouts_match_header(cv, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cvib.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(cv_pair),'
                   ' sizeof(cv_color_summary), sizeof(cv_table_row), sizeof(cv_grid),'
                   ' sizeof(cv_rule), offsetof(cv_color_summary, per_pattern),'
                   ' offsetof(cv_pair, flags), sizeof(cv_pattern_pair));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals[0] == cv.PAIR_DTYPE.itemsize == 16
    assert vals[1] == cv.SUMMARY_DTYPE.itemsize == 48
    assert vals[2] == cv.TABLE_DTYPE.itemsize == 40
    assert vals[3] == C.sizeof(cv.cv_grid) and vals[4] == C.sizeof(cv.cv_rule)
    assert vals[5] == cv.SUMMARY_DTYPE.fields["per_pattern"][1]
    assert vals[6] == cv.PAIR_DTYPE.fields["flags"][1]
    assert vals[7] == cv.PATTERN_PAIR_DTYPE.itemsize == 12


def test_null_context_is_rejected(cv):
    L = cv.lib()
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule().c()
    tot = C.c_int64(0)
    assert L.cv_lab_convert(None, None, None, 0, 0, None) == cv.CV_EINVAL
    assert b"ctx" in L.cv_last_error()
    assert L.cv_pair_search(None, None, 0, C.byref(g), C.byref(r), None, 0, None, None,
                            C.byref(tot), 0, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce(None, None, 0, C.byref(g), C.byref(r), None, None, None) == cv.CV_EINVAL
    assert L.cv_frames_resolve(None, None, 1, None, C.byref(g), C.byref(r), None, 1, None, None,
                               None, None, None, None, None, None, 0, None) == cv.CV_EINVAL
    assert L.cv_context_destroy(None) == cv.CV_OK
    assert L.cv_context_create(0, None) == cv.CV_EINVAL
    assert L.cv_context_set_timing(None, 1) == cv.CV_EINVAL


@pytest.mark.parametrize("grid,ok", [
    ((0.1, 10, 1.0, 360), True),
    ((0.0, 10, 1.0, 360), False),      # dr must be > 0
    ((0.1, 0, 1.0, 360), False),       # nr >= 1
    ((0.1, 10, 1.0, 361), False),      # ntheta beyond one turn
    ((0.1, 10, 7.0, 10), False),       # 360/7 not an integer
    ((0.1, 10, 120.0, 3), False),      # 360/120 = 3 is odd
    ((0.1, 65536, 1.0, 10), False),    # nr too large
    ((0.1, 60000, 0.01, 36000), False),  # nr * ntheta >= 2^31
])
def test_grid_validation(cv, grid, ok):
    """Grid and rule checks run before the context is used (a dummy context
    buffer stands in, so no device is touched)."""
    L = cv.lib()
    dummy = (C.c_uint8 * 4096)()
    g = cv.Grid(*grid).c()
    r = cv.Rule().c()
    tot = C.c_int64(0)
    if ok:
        return  # a valid grid would proceed to the device
    rc = L.cv_pair_search(C.cast(dummy, C.c_void_p), None, 0, C.byref(g), C.byref(r), None, 0,
                          None, None, C.byref(tot), 0, None)
    assert rc == cv.CV_EINVAL, L.cv_last_error()


@pytest.mark.parametrize("rule", [(0, 0.5, 0x7F), (256, 0.5, 0x7F), (50, 0.0, 0x7F),
                                  (50, 1.0, 0x7F), (50, 0.5, 0x80), (50, 0.5, 0x7F, 2)])
def test_rule_validation(cv, rule):
    L = cv.lib()
    dummy = (C.c_uint8 * 4096)()
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule(*rule).c()
    tot = C.c_int64(0)
    rc = L.cv_pair_search(C.cast(dummy, C.c_void_p), None, 0, C.byref(g), C.byref(r), None, 0,
                          None, None, C.byref(tot), 0, None)
    assert rc == cv.CV_EINVAL


def test_argument_validation(cv):
    L = cv.lib()
    dummy = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule().c()
    tot = C.c_int64(0)
    # negative capacity, capacity without an output array, neither total nor offsets
    assert L.cv_pair_search(dummy, None, 0, C.byref(g), C.byref(r), None, -1, None, None,
                            C.byref(tot), 0, None) == cv.CV_EINVAL
    assert L.cv_pair_search(dummy, None, 0, C.byref(g), C.byref(r), None, 5, None, None,
                            C.byref(tot), 0, None) == cv.CV_EINVAL
    assert L.cv_pair_search(dummy, None, 0, C.byref(g), C.byref(r), None, 0, None, None,
                            None, 0, None) == cv.CV_EINVAL
    assert L.cv_pair_search(dummy, None, 0, C.byref(g), C.byref(r), None, 0, None, None,
                            C.byref(tot), 0x80, None) == cv.CV_EINVAL
    assert L.cv_pair_search(dummy, None, 3, C.byref(g), C.byref(r), None, 0, None, None,
                            C.byref(tot), 0, None) == cv.CV_EINVAL  # rgb NULL with n > 0
    assert L.cv_lab_convert(dummy, None, None, 4, 0, None) == cv.CV_EINVAL
    assert L.cv_lab_convert(dummy, None, None, 0, 7, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce(dummy, None, 0, C.byref(g), C.byref(r), None, None, None) == cv.CV_EINVAL
    gbig = cv.Grid(0.1, 300, 1.0, 360).c()
    assert L.cv_pair_reduce(dummy, None, 0, C.byref(gbig), C.byref(r), None,
                            C.cast(dummy, C.c_void_p), None) == cv.CV_EINVAL  # table needs nr<=255


def test_frames_argument_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule().c()

    def call(npix=4, colour_cap=4, fa=d, fb=d, res=None, flags=0, pixels=d, pbest=d):
        return L.cv_frames_resolve(d, pixels, npix, None, C.byref(g), C.byref(r), d, colour_cap, d,
                                   d, None, pbest, None, fa, fb, res, flags, None)
    assert call(npix=0) == cv.CV_EINVAL                # no pixels
    assert call(pixels=None) == cv.CV_EINVAL           # null input
    assert call(pbest=None) == cv.CV_EINVAL            # pbest is required
    assert call(colour_cap=3) == cv.CV_EINVAL          # fewer slots than possible colours
    assert b"colour_cap" in L.cv_last_error()
    assert call(fb=None) == cv.CV_EINVAL               # the two frames go together
    assert call(fa=None, fb=None, res=d) == cv.CV_EINVAL
    assert call(flags=0x20) == cv.CV_EINVAL            # unknown flag


def test_frames_generate_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    seeds = (C.c_uint64 * 2)(1, 2)

    def call(ctx=d, sd=seeds, n=1, h=4, w=4, sites=8, noise=4, out=d):
        return L.cv_frames_generate(ctx, sd, n, h, w, sites, noise, out, None)
    assert call(ctx=None) == cv.CV_EINVAL
    assert call(sd=None) == cv.CV_EINVAL
    assert call(out=None) == cv.CV_EINVAL
    assert call(n=-1) == cv.CV_EINVAL
    for h, w in ((0, 4), (4, 0), (16385, 4), (4, 16385)):
        assert call(h=h, w=w) == cv.CV_EINVAL
    for sites in (0, 257):
        assert call(sites=sites) == cv.CV_EINVAL
    for noise in (-1, 256):
        assert call(noise=noise) == cv.CV_EINVAL
    assert b"noise" in L.cv_last_error()


def test_best_pair_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule().c()
    assert L.cv_best_pair_search(None, d, 4, C.byref(g), C.byref(r), d, d, None, None) == cv.CV_EINVAL
    assert L.cv_best_pair_search(d, d, 4, C.byref(g), C.byref(r), None, None, None, None) == cv.CV_EINVAL
    assert L.cv_best_pair_search(d, None, 4, C.byref(g), C.byref(r), d, None, None, None) == cv.CV_EINVAL
    assert L.cv_best_pair_search(d, d, -1, C.byref(g), C.byref(r), d, None, None, None) == cv.CV_EINVAL
    gbad = cv.Grid(0.1, 10, 7.0, 360).c()   # 360 / 7 is not an integer
    assert L.cv_best_pair_search(d, d, 4, C.byref(gbad), C.byref(r), d, None, None, None) == cv.CV_EINVAL


def test_binding_refuses_host_tensors(cv):
    import torch
    with pytest.raises(ValueError):
        cv.pair_search(torch.zeros((2, 3), dtype=torch.uint8), cv.Grid(0.1, 10, 1.0, 360), cv.Rule())
    with pytest.raises(ValueError):
        cv.rgb8_to_lab(torch.zeros((2, 4), dtype=torch.uint8))


def test_mlp_argument_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    h = C.c_void_p()

    def create(dims):
        arr = (C.c_int32 * len(dims))(*dims)
        return L.cv_mlp_create(d, arr, len(dims) - 1, C.byref(h))
    arr = (C.c_int32 * 5)(3, 256, 256, 256, 37)
    assert L.cv_mlp_create(None, arr, 4, C.byref(h)) == cv.CV_EINVAL
    assert create([3, 37]) == cv.CV_EINVAL                 # one layer
    assert create([4, 64, 37]) == cv.CV_EINVAL             # not an RGB input
    assert create([3, 48, 37]) == cv.CV_EINVAL             # width not a multiple of 32
    assert create([3, 2048, 37]) == cv.CV_EINVAL           # too wide
    assert create([3, 64, 300]) == cv.CV_EINVAL            # output too wide
    assert create([3] + [32] * 9 + [37]) == cv.CV_EINVAL   # too deep
    assert L.cv_mlp_destroy(None) == cv.CV_OK
    assert L.cv_mlp_forward(None, None, 0, None, 0, None) == cv.CV_EINVAL
    assert L.cv_mlp_loss(None, None, None, None, 1, 0.1, None, None, None) == cv.CV_EINVAL
    assert L.cv_mlp_backward(None, None, None, 1, None) == cv.CV_EINVAL
    assert L.cv_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, 1, None) == cv.CV_EINVAL
    assert L.cv_mlp_save(None, b"/tmp/x") == cv.CV_EINVAL
    assert L.cv_mlp_load(None, b"/tmp/x") == cv.CV_EINVAL
    assert L.cv_mlp_set_first_sine(None, 30.0) == cv.CV_EINVAL
    assert L.cv_mlp_first_sine(None, None) == cv.CV_EINVAL
    assert L.cv_permute_ids(None, None, 1, 0, None, None) == cv.CV_EINVAL


def test_init_params_layout(cv):
    dims = cv.SURROGATE_DIMS
    flat = cv.init_params(dims, 0)
    assert flat.dtype == np.float32 and flat.size == 142117
    Ws, bs = cv.split_params(flat, dims)
    assert [w.shape for w in Ws] == [(256, 3), (256, 256), (256, 256), (37, 256)]
    assert all(np.all(b == 0) for b in bs)
    assert abs(Ws[1].std() - np.sqrt(2 / 256)) < 0.01
    # a sinusoidal first layer starts uniform; the other layers as before
    fs = cv.init_params(dims, 0, first_sine=True)
    Ws2, bs2 = cv.split_params(fs, dims)
    assert np.all(np.abs(Ws2[0]) <= 1 / 3) and Ws2[0].std() > 0.15
    assert np.all(np.abs(bs2[0]) <= 3 ** -0.5) and bs2[0].std() > 0.25
    assert abs(Ws2[1].std() - np.sqrt(2 / 256)) < 0.01 and all(np.all(b == 0) for b in bs2[1:])


def test_resolve_variant_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    assert L.cv_context_set_autotune(None, 1) == cv.CV_EINVAL
    assert L.cv_context_set_resolve_variant(None, 0) == cv.CV_EINVAL
    assert L.cv_context_set_resolve_variant(d, 3) == cv.CV_EINVAL
    assert L.cv_context_set_resolve_variant(d, -2) == cv.CV_EINVAL
    v = C.c_int(0)
    assert L.cv_context_resolve_variant(None, None, 0, C.byref(v), None) == cv.CV_EINVAL


def test_tuner_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    assert L.cv_context_set_tile_target(None, 0) == cv.CV_EINVAL
    assert L.cv_context_set_tile_target(d, 5) == cv.CV_EINVAL
    assert L.cv_context_set_tile_target(d, (1 << 20) + 1) == cv.CV_EINVAL
    t = C.c_int32(0)
    assert L.cv_context_tile_target(None, 1, None, 1, C.byref(t), None) == cv.CV_EINVAL
    assert L.cv_context_tile_target(d, 1, None, 1, None, None) == cv.CV_EINVAL
    assert L.cv_context_set_tune_file(None, b"tune.txt") == cv.CV_EINVAL


def test_rules_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    rules = (cv.cv_rule * 17)(*[cv.Rule().c() for _ in range(17)])
    assert L.cv_pair_reduce_rules(None, d, 1, C.byref(g), C.cast(rules, C.c_void_p), 1, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_rules(d, d, 1, C.byref(g), C.cast(rules, C.c_void_p), 0, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_rules(d, d, 1, C.byref(g), C.cast(rules, C.c_void_p), 17, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_rules(d, d, 1, C.byref(g), None, 3, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_rules(d, None, 1, C.byref(g), C.cast(rules, C.c_void_p), 3, d, None) == cv.CV_EINVAL


def test_per_ray_and_list_validation(cv):
    L = cv.lib()
    d = C.cast((C.c_uint8 * 4096)(), C.c_void_p)
    g = cv.Grid(0.1, 10, 1.0, 360).c()
    r = cv.Rule().c()
    tot = C.c_int64(0)
    both = cv.CV_EMIT_ALL | cv.CV_PER_RAY
    assert L.cv_pair_search(d, d, 1, C.byref(g), C.byref(r), None, 0, None, None, C.byref(tot), both,
                            None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_csr(None, d, d, 1, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_csr(d, d, None, 1, d, None) == cv.CV_EINVAL
    assert L.cv_pair_reduce_csr(d, d, d, -1, d, None) == cv.CV_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message, before
    touching a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
