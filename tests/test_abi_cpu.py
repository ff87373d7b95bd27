"""Host-only checks of the C ABI: the library loads without a GPU, exports
every entry point include/posegraph.h declares, the ctypes structures match
the C layout, and argument checking answers before any device is touched."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "posegraph.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def lib():
    from paper_2108_00516_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2108_00516_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:pose_graph|pg)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "pose_graph_optimize" in names and "pose_graph_create" in names
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    from paper_2108_00516_amd import _lib
    assert sorted(_lib.SIGNATURES) == names


def test_struct_layout_matches_c(lib):
    from paper_2108_00516_amd import _lib
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "posegraph.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(pg_camera), sizeof(pg_config), sizeof(pg_stats));
  printf("%zu %zu %zu %zu\n", offsetof(pg_config, solver), offsetof(pg_config, prune_frac),
         offsetof(pg_stats, status_bits), offsetof(pg_stats, ms_total));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert vals[:3] == [C.sizeof(_lib.pg_camera), C.sizeof(_lib.pg_config), C.sizeof(_lib.pg_stats)]
    assert vals[3:] == [_lib.pg_config.solver.offset, _lib.pg_config.prune_frac.offset,
                        _lib.pg_stats.status_bits.offset, _lib.pg_stats.ms_total.offset]


def test_defaults(lib):
    from paper_2108_00516_amd import Config, _lib
    c = _lib.pg_config()
    lib.pg_config_default(C.byref(c))
    py = Config()
    for name, _ in _lib.pg_config._fields_:
        assert getattr(c, name) == pytest.approx(getattr(py, name)), name


def test_argument_checks_without_device(lib):
    from paper_2108_00516_amd import _lib
    cfg = _lib.pg_config()
    lib.pg_config_default(C.byref(cfg))
    out = C.c_void_p()
    cam = _lib.pg_camera(2, 480, 615.0, 615.0, 320.0, 240.0)   # width too small
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_INVALID_ARG
    assert b"image size" in lib.pose_graph_last_error(None)
    cam = _lib.pg_camera(640, 480, -1.0, 615.0, 320.0, 240.0)
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_INVALID_ARG
    cam = _lib.pg_camera(640, 480, 615.0, 615.0, 320.0, 240.0)
    cfg.max_frames = 33
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_INVALID_ARG
    lib.pg_config_default(C.byref(cfg))
    cfg.gn_iters = 33
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_INVALID_ARG
    lib.pg_config_default(C.byref(cfg))
    cfg.huber_g_m = 0.0
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_INVALID_ARG
    assert out.value is None
    # NULL handles are rejected and destroy(NULL) is a no-op
    assert lib.pose_graph_optimize(None, None) == _lib.PG_ERR_INVALID_ARG
    assert lib.pose_graph_num_frames(None) == 0
    lib.pose_graph_destroy(None)


def test_no_device_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2108_00516_amd import _lib
    cfg = _lib.pg_config()
    lib.pg_config_default(C.byref(cfg))
    cam = _lib.pg_camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    out = C.c_void_p()
    assert lib.pose_graph_create(C.byref(cfg), C.byref(cam), None, C.byref(out)) == _lib.PG_ERR_NO_DEVICE


def test_match_argument_errors_without_a_device(lib):
    """pg_match_descriptors checks sizes before it touches the device."""
    from paper_2108_00516_amd import _lib
    off = (C.c_int * 3)(0, 5, 10)
    pa = (C.c_int * 97)(*([0] * 97))
    pb = (C.c_int * 97)(*([1] * 97))
    args = lambda n_pairs, dim, ratio: (None, off, 2, dim, pa, pb, n_pairs, ratio, None, None, None, None)
    assert lib.pg_match_descriptors(*args(0, 128, 1.0)) == _lib.PG_ERR_INVALID_ARG
    assert lib.pg_match_descriptors(*args(97, 128, 1.0)) == _lib.PG_ERR_CAPACITY
    assert lib.pg_match_descriptors(*args(1, 100, 1.0)) == _lib.PG_ERR_INVALID_ARG
    assert lib.pg_match_descriptors(*args(1, 128, -1.0)) == _lib.PG_ERR_INVALID_ARG
    assert lib.pg_frontend_last_error()


def test_tile_table_argument_checks(lib):
    """pg_set_tile_table validates every record (positive resolution, a
    node range, a tile that is a multiple of 256 in 256..2048) and the count,
    before anything changes; a valid table and an empty one are accepted."""
    from paper_2108_00516_amd import _lib, autotune

    def call(rows):
        arr = (C.c_int * (5 * max(len(rows), 1)))(*[v for r in rows for v in r])
        return lib.pg_set_tile_table(arr, len(rows))
    try:
        assert call([(640, 480, 8, 11, 768), (320, 240, 2, 7, 256)]) == 0
        for bad in [(0, 480, 8, 11, 768), (640, 480, 0, 11, 768), (640, 480, 9, 8, 768),
                    (640, 480, 8, 11, 700), (640, 480, 8, 11, 128), (640, 480, 8, 11, 2304)]:
            assert call([bad]) == _lib.PG_ERR_INVALID_ARG, bad
            assert b"tile table" in lib.pose_graph_last_error(None)
        assert lib.pg_set_tile_table(None, 1) == _lib.PG_ERR_INVALID_ARG
        assert lib.pg_set_tile_table(None, 257) == _lib.PG_ERR_INVALID_ARG
        assert lib.pg_set_tile_table(None, 0) == 0
        # the class keys of the autotuner's table map onto the records
        assert autotune.table_entries({"640x480/8-11": {"tile": 768}, "batch": {"tile": 1024},
                                       "320x240/other": {"tile": 512}}) == [(640, 480, 8, 11, 768)]
    finally:
        table = autotune.load(autotune.TABLE_PATH)
        if table:
            autotune.apply(table, lib)
        else:
            lib.pg_set_tile_table(None, 0)
