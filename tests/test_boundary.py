"""The C-ABI library loads and exports every function include/edt.h declares.

CPU-only: the library is opened and its symbols resolved; the only calls
made are ones that return from host-side argument validation before any
HIP call (bad grids, NULL pointers), plus the pure string helpers.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\**\s+\**([a-z_][a-z0-9_]*)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_02363_amd import edt
    if not os.path.exists(edt.LIB_PATH):
        pytest.fail("libedtmi.so not built (run __graft_entry__.build())")
    return edt.lib()


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for n in ["edt_insert_points", "edt_insert_links", "edt_compute", "edt_query_spheres"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_struct_sizes_match_header():
    from paper_2407_02363_amd import edt
    assert ctypes.sizeof(edt.SphereResult) == 64
    assert ctypes.sizeof(edt.EdtGrid) == 28


def test_status_strings(lib):
    assert lib.edt_status_string(0) == b"ok"
    assert lib.edt_status_string(-2) == b"invalid grid shape"
    assert b"gfx950" in lib.edt_version()


def test_host_validation_rejects_bad_arguments(lib):
    from paper_2407_02363_amd import edt
    bad = edt.EdtGrid(0, 4, 4, (ctypes.c_float * 3)(0, 0, 0), 0.01)
    rc = lib.edt_compute(ctypes.byref(bad), None, None, None, None, 0, None)
    assert rc == -2 and b"outside" in lib.edt_last_error()
    big = edt.EdtGrid(1025, 4, 4, (ctypes.c_float * 3)(0, 0, 0), 0.01)
    assert lib.edt_compute(ctypes.byref(big), None, None, None, None, 0, None) == -2
    nanv = edt.EdtGrid(4, 4, 4, (ctypes.c_float * 3)(0, 0, 0), float("nan"))
    assert lib.edt_compute(ctypes.byref(nanv), None, None, None, None, 0, None) == -2
    ok = edt.EdtGrid(4, 4, 4, (ctypes.c_float * 3)(0, 0, 0), 0.01)
    assert lib.edt_compute(ctypes.byref(ok), None, None, None, None, 0, None) == -1
    assert lib.edt_compute(None, None, None, None, None, 0, None) == -1
    assert lib.edt_insert_points(ctypes.byref(ok), None, None, -1, None, None, None) == -1
    off = (ctypes.c_int32 * 2)(1, 5)
    assert lib.edt_insert_links(ctypes.byref(ok), ctypes.c_void_p(16), None, off, 1,
                                ctypes.c_void_p(16), 1, None) == -1
    assert lib.edt_query_spheres(ctypes.byref(ok), None, None, None, None, -3, None, None) == -1
    # zero-sized requests are accepted without launching anything
    assert lib.edt_insert_points(ctypes.byref(ok), None, None, 0, None, None, None) == 0
    assert lib.edt_query_spheres(ctypes.byref(ok), None, None, None, None, 0, None, None) == 0
    assert lib.edt_workspace_bytes(ctypes.byref(ok)) == 0
    # tuning: defaults are valid tiles; bad tiles are rejected before launch
    one = ctypes.c_void_p(256)
    t = edt.Tuning()
    assert lib.edt_default_tuning(ctypes.byref(ok), ctypes.byref(t)) == 0
    assert t.xy_tile in (16, 32, 64) and t.z_tile in (8, 16, 32, 64) and t.z_group in (64, 128, 256)
    assert lib.edt_compute_tuned(ctypes.byref(ok), one, one, one, ctypes.byref(edt.Tuning(32, 64, 32)),
                                 None) == -5
    bad_t = edt.Tuning(24, 8)
    assert lib.edt_compute_tuned(ctypes.byref(ok), one, one, one, ctypes.byref(bad_t), None) == -5
    # edt_compute_many: map count, NULL buffers and tiles are checked before any launch
    maps = (edt.BatchMap * 49)()
    for m in maps:
        m.grid, m.occ, m.d2, m.site = ok, 256, 256, 256
    assert lib.edt_compute_many(ctypes.cast(maps, ctypes.c_void_p), 0, None, None) == -1
    assert lib.edt_compute_many(ctypes.cast(maps, ctypes.c_void_p), 49, None, None) == -1
    assert lib.edt_compute_many(ctypes.cast(maps, ctypes.c_void_p), 2, ctypes.byref(bad_t), None) == -5
    maps[1].d2 = None
    assert lib.edt_compute_many(ctypes.cast(maps, ctypes.c_void_p), 2, ctypes.byref(bad_t), None) == -1
    # log-odds update: workspace size, clamp range and NULLs, before any launch
    assert lib.edt_logodds_workspace_bytes(ctypes.byref(ok)) >= 2 * ok.nx * ok.ny * ok.nz
    lo = edt.LogOdds(85, -41, 10, -10, 0, 0)
    wsb = lib.edt_logodds_workspace_bytes(ctypes.byref(ok))
    assert lib.edt_update_logodds(ctypes.byref(ok), one, one, one, 1, one, None, None,
                                  ctypes.byref(lo), one, wsb, None) == -1
    lo = edt.LogOdds(*edt.LOGODDS_DEFAULT, 0)
    assert lib.edt_update_logodds(ctypes.byref(ok), one, one, one, 1, one, None, None,
                                  ctypes.byref(lo), one, wsb - 1, None) == -3
    assert lib.edt_update_logodds(ctypes.byref(ok), one, None, one, 1, one, None, None,
                                  ctypes.byref(lo), one, wsb, None) == -1
    # outlier filter: k, radius, point count and workspace before any launch
    ow = lib.edt_outlier_workspace_bytes(1000)
    assert ow > 16 * 1000 and lib.edt_outlier_workspace_bytes(edt.OUTLIER_MAX_POINTS + 1) == 0
    assert lib.edt_outlier_filter(one, 1000, 0, 0.01, 1.0, one, None, None, one, ow, None) == -1
    assert lib.edt_outlier_filter(one, 1000, 17, 0.01, 1.0, one, None, None, one, ow, None) == -1
    assert lib.edt_outlier_filter(one, 1000, 8, 0.0, 1.0, one, None, None, one, ow, None) == -1
    assert lib.edt_outlier_filter(one, 1000, 8, 0.01, float("nan"), one, None, None, one, ow,
                                  None) == -1
    assert lib.edt_outlier_filter(one, 1000, 8, 0.01, 1.0, one, None, None, one, ow - 1, None) == -3
    assert lib.edt_outlier_filter(one, -1, 8, 0.01, 1.0, one, None, None, one, ow, None) == -1
    # the exact fixed-point sums bound n * radius^2 (d_i <= radius)
    owm = lib.edt_outlier_workspace_bytes(1_000_000)
    assert lib.edt_outlier_filter(one, 1_000_000, 8, 0.2, 1.0, one, None, None, one, owm, None) == -1
    assert b"overflow" in lib.edt_last_error()
    ow4 = lib.edt_outlier_workspace_bytes(edt.OUTLIER_MAX_POINTS)
    assert lib.edt_outlier_filter(one, edt.OUTLIER_MAX_POINTS, 8, 0.09, 1.0, one, None, None, one, ow4,
                                  None) == -1
    # cached transform: cache size and NULLs before any launch
    cb = lib.edt_cache_workspace_bytes(ctypes.byref(ok))
    assert cb >= 256 + ok.nx * ok.ny * ok.nz
    assert lib.edt_compute_cached(ctypes.byref(ok), one, one, one, one, cb - 1, None) == -3
    assert lib.edt_compute_cached(ctypes.byref(ok), one, None, one, one, cb, None) == -1
    assert lib.edt_cache_reset(ctypes.byref(ok), one, cb - 1, None) == -3
    assert lib.edt_logodds_reset(ctypes.byref(ok), one, one, 16, None) == -3
    huge = edt.EdtGrid(8, 1024, 8, (ctypes.c_float * 3)(0, 0, 0), 0.01)
    assert lib.edt_compute_tuned(ctypes.byref(huge), one, one, one,
                                 ctypes.byref(edt.Tuning(64, 8)), None) == -5
    assert lib.edt_compute_stage(ctypes.byref(ok), one, one, one, 4, None, None) == -1
    assert lib.edt_autotune(ctypes.byref(ok), one, one, one, 0, None, None, None) == -1


CACHE_LINES = ["single gfx950 256 256 128 xy 64 512 z 64 256",
               "batch gfx950 32 256 256 128 xy 64 256 z 64 256",
               "single gfx942 512 512 512 xy 32 512 z 16 256"]


def test_tuning_cache_file_round_trip(lib, tmp_path):
    """The autotuners' cache is written to and read from a text file on the
    host: a saved file holds exactly the loaded entries, a reloaded one gives
    them back, and a file with any invalid line adds nothing."""
    from paper_2407_02363_amd import edt
    edt.edt_tuning_cache_clear()
    src = tmp_path / "cache.txt"
    src.write_text("edtmi tuning cache v1\n# tiles per architecture\n" + CACHE_LINES[0] + "\n\n" +
                   "\n".join(CACHE_LINES[1:]) + "\n")
    assert edt.edt_tuning_cache_load(src) == 3
    out = tmp_path / "saved.txt"
    assert edt.edt_tuning_cache_save(out) == 3
    lines = out.read_text().splitlines()
    assert lines[0] == "edtmi tuning cache v1" and sorted(lines[1:]) == sorted(CACHE_LINES)
    edt.edt_tuning_cache_clear()
    empty = tmp_path / "empty.txt"
    assert edt.edt_tuning_cache_save(empty) == 0
    assert empty.read_text() == "edtmi tuning cache v1\n"
    assert edt.edt_tuning_cache_load(out) == 3
    bad = {
        "header": "edtmi tuning cache v2\n" + CACHE_LINES[0] + "\n",
        "xy tile": "edtmi tuning cache v1\nsingle gfx950 256 256 128 xy 128 512 z 64 256\n",
        "z group": "edtmi tuning cache v1\nsingle gfx950 256 256 128 xy 64 512 z 64 1024\n",
        "grid": "edtmi tuning cache v1\nsingle gfx950 0 256 128 xy 64 512 z 64 256\n",
        "maps": "edtmi tuning cache v1\nbatch gfx950 49 256 256 128 xy 32 256 z 64 256\n",
        "batch tile": "edtmi tuning cache v1\nbatch gfx950 4 256 256 128 xy 64 256 z 32 256\n",
        "trailing": "edtmi tuning cache v1\nsingle gfx950 256 256 128 xy 64 512 z 64 256 7\n",
        "short": "edtmi tuning cache v1\nsingle gfx950 256 256 xy 64 512 z 64 256\n",
        "kind": "edtmi tuning cache v1\ndouble gfx950 256 256 128 xy 64 512 z 64 256\n",
        "empty": "",
    }
    for name, text in bad.items():
        f = tmp_path / f"bad_{name.replace(' ', '_')}.txt"
        # a valid line after the invalid one must not be added either
        good_then_bad = text if name in ("header", "empty") else text + CACHE_LINES[1] + "\n"
        f.write_text(good_then_bad)
        edt.edt_tuning_cache_clear()
        with pytest.raises(edt.EdtError):
            edt.edt_tuning_cache_load(f)
        assert edt.edt_tuning_cache_save(empty) == 0, name
    with pytest.raises(edt.EdtError):
        edt.edt_tuning_cache_load(tmp_path / "missing.txt")
    edt.edt_tuning_cache_clear()
