"""CPU-side checks of the C ABI: the built library loads and exports every
function include/fpm.h declares (no compute call needs a GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1711_08475_amd", "libfpm.so")


def declared(header: str):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared("fpm.h")
    for n in ["fpm_build_fingerprints", "fpm_match", "fpm_plan_create", "fpm_plan_run", "fpm_plan_result",
              "fpm_select_symbols", "fpm_verify_pairs", "fpm_autotune"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfpm.so not built")
@pytest.mark.parametrize("header", ["fpm.h", "fpm_learn.h", "fpm_peak.h"])
def test_library_exports_every_declared_symbol(header):
    lib = ctypes.CDLL(LIB)
    names = declared(header)
    assert names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfpm.so not built")
def test_binding_names_match_header():
    from paper_1711_08475_amd import fpm

    assert sorted(fpm.EXPORTS) == declared("fpm.h")
    assert sorted(fpm.LEARN_EXPORTS) == declared("fpm_learn.h")
    assert sorted(fpm.PEAK_EXPORTS) == declared("fpm_peak.h")
    for n in fpm.EXPORTS + fpm.LEARN_EXPORTS + fpm.PEAK_EXPORTS:
        if n in ("fpm_last_error", "fpm_free", "fpm_index_destroy", "fpm_plan_destroy"):
            continue
        assert callable(getattr(fpm, n)), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfpm.so not built")
def test_num_fields_without_gpu():
    from paper_1711_08475_amd import fpm

    assert [fpm.fpm_num_fields(v, 16) for v in ("occ", "count", "pos", "occh")] == [16, 8, 6, 8]
    assert [fpm.fpm_num_fields(v, 32) for v in ("occ", "count", "pos", "occh")] == [32, 16, 12, 16]
    assert fpm.fpm_num_fields("qgram", 16) == 16 and fpm.fpm_num_fields("qgram", 32) == 32
    assert fpm.fpm_num_fields("combo", 16) == 8 and fpm.fpm_num_fields("combo", 32) == 16
    assert fpm.fpm_num_fields(6, 16) == -1
    assert fpm.fpm_num_fields("occ", 8) == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with a message before any
    device work."""
    import subprocess
    import sys as _sys

    r = subprocess.run([_sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_roofline_follows_the_filter_unit():
    """The bench prices the match kernel with the VALU work of the unit that
    ran the filter (fpm_stats.filter_unit): 3 ops per examined occ16 pair on
    the vector ALUs, 1 (the sign-bit shift) on the matrix cores, where the
    int8 contraction (64 ops per pair) is reported against the matrix peak."""
    import sys as _sys

    _sys.path.insert(0, ROOT)
    import bench
    from paper_1711_08475_amd import fpm as f

    st = {"pairs_examined": 1_000_000, "verify_cells": 500_000, "filter_unit": f.FPM_UNIT_VALU}
    r = bench.roofline_of(st, 0.001, "occ", 16, None)
    assert r["filter_unit"] == "valu" and r["valu_ops_per_pair"] == 3
    assert r["ops_per_launch"] == 3_500_000
    assert abs(r["achieved"] - 3.5e6 / 1e-6 / 1e12) < 1e-9
    assert abs(r["frac"] - 3.5e12 / (256 * 64 * 2.4e9)) < 1e-12
    assert "matrix_cores" not in r and r["traffic"] is None and r["bound"] == "alu"
    st["filter_unit"] = f.FPM_UNIT_MATRIX
    r = bench.roofline_of(st, 0.001, "occ", 16, {"bytes_per_launch": 123})
    assert r["filter_unit"] == "matrix" and r["valu_ops_per_pair"] == 1
    assert r["ops_per_launch"] == 1_500_000 and r["traffic"] == 123
    assert abs(r["matrix_cores"]["frac"] - 64e6 / 1e-6 / 5.0e15) < 1e-12
    r = bench.roofline_of(st, 0.001, "occ", 16, None, {"int_valu_ops_per_s": 4.0e13,
                                                        "int8_matrix_ops_per_s": 4.5e15})
    assert abs(r["peak_measured"] - 40.0) < 1e-9 and abs(r["matrix_cores"]["peak_measured"] - 4500.0) < 1e-9
    assert abs(r["peak"] - 39.3216) < 1e-9  # the published peak stays the reference
    # no kernel time: nothing achieved, nothing divided by zero
    r = bench.roofline_of(st, None, "occ", 16, None)
    assert r["achieved"] is None and r["frac"] is None and "matrix_cores" not in r
