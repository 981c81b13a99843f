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


def test_bench_roofline_prices_the_methods_work():
    """The bench prices the match kernel with the method's algorithmic work,
    whichever unit ran the filter test: filter ops per examined pair (occ 3,
    count16 3, count32 5, pos 9) x examined pairs + (2k+1) min(m, n) band
    cells of the survivors, over the kernel's duration, against the published
    int-VALU peak (with popcount pruning, the pricing over the pairs the
    filter tested beside it).  Issued-VALU utilisation and the matrix-core
    int8 fraction are reported beside it under their own names."""
    import sys as _sys

    _sys.path.insert(0, ROOT)
    import bench
    from paper_1711_08475_amd import fpm as f

    assert [bench.filter_ops(v, b) for v, b in [("occ", 16), ("occ", 32), ("count", 16), ("count", 32),
                                                 ("pos", 16), ("occh", 16), ("qgram", 32), ("combo", 32)]] == \
        [3, 3, 3, 5, 9, 3, 3, 6]
    # 1M English-like words x 10K queries, learned occ16, Lev k = 1: 4.186e9
    # examined pairs, 2.321e9 band cells, match kernel 0.5894 ms (matrix
    # cores ran the filter): 1.488e10 ops / 0.5894 ms / 39.32 Tops/s = 0.64
    st = {"pairs_examined": 4_186_148_656, "verify_cells": 2_321_000_000, "filter_unit": f.FPM_UNIT_MATRIX}
    r = bench.roofline_of(st, 0.5894, "occ", 16, None)
    assert r["filter_unit"] == "matrix" and r["filter_ops_per_pair"] == 3
    assert r["ops_per_launch"] == 3 * 4_186_148_656 + 2_321_000_000
    assert abs(r["frac"] - 0.642) < 0.002
    assert abs(r["matrix_cores"]["frac"] - 64 * 4_186_148_656 / 0.5894e-3 / 5.0e15) < 1e-12
    st["filter_unit"] = f.FPM_UNIT_VALU
    r2 = bench.roofline_of(st, 0.5894, "occ", 16, {"bytes_per_launch": 123, "valu_insts_per_launch": 2.93e8},
                           hbm_bytes=19_000_000)
    assert r2["frac"] == r["frac"] and "matrix_cores" not in r2 and r2["traffic"] == 123
    assert abs(r2["valu_issue"]["utilisation"] - 2.93e8 / (256 * 4 * 2.4e9 / 4 * 0.5894e-3)) < 1e-12
    assert abs(r2["hbm"]["frac"] - 19e6 / 0.5894e-3 / 8e12) < 1e-12
    st = {"pairs_examined": 1_000_000, "verify_cells": 500_000, "filter_unit": f.FPM_UNIT_VALU}
    r = bench.roofline_of(st, 0.001, "count", 32, None)
    assert r["ops_per_launch"] == 5_500_000 and r["bound"] == "alu"
    assert abs(r["achieved"] - 5.5e6 / 1e-6 / 1e12) < 1e-9
    r = bench.roofline_of(st, 0.001, "occ", 16, None, {"int_valu_ops_per_s": 4.0e13,
                                                        "int8_matrix_ops_per_s": 4.5e15})
    assert abs(r["peak_measured"] - 40.0) < 1e-9
    assert abs(r["peak"] - 39.3216) < 1e-9  # the published peak stays the reference
    # no kernel time: nothing achieved, nothing divided by zero
    r = bench.roofline_of(st, None, "occ", 16, None)
    assert r["achieved"] is None and r["frac"] is None and "matrix_cores" not in r
    # popcount pruning: the method's work stays priced per examined pair; the
    # pricing over the pairs the filter tested is reported beside it
    st = {"pairs_examined": 1_000_000, "pairs_filtered": 800_000, "verify_cells": 500_000,
          "filter_unit": f.FPM_UNIT_VALU}
    r = bench.roofline_of(st, 0.001, "occ", 32, None)
    assert r["ops_per_launch"] == 3 * 1_000_000 + 500_000 and r["pairs_tested"] == 800_000
    assert abs(r["frac_tested"] - 2.9e6 / 1e-6 / bench.PEAK_INT_OPS) < 1e-12
    st["pairs_filtered"] = 1_000_000
    assert "frac_tested" not in bench.roofline_of(st, 0.001, "occ", 32, None)


STRUCTS = {  # header type -> binding class, header file
    "fpm_hit": ("Hit", "fpm.h"),
    "fpm_stats": ("Stats", "fpm.h"),
    "fpm_options": ("Options", "fpm.h"),
    "fpm_peaks": ("Peaks", "fpm_peak.h"),
    "fpm_learn_config": ("LearnConfig", "fpm_learn.h"),
    "fpm_learn_report": ("LearnReport", "fpm_learn.h"),
}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Size and every field offset of the ctypes structures equal what a C
    compiler lays out from include/*.h (gcc on the host)."""
    import shutil
    import subprocess

    from paper_1711_08475_amd import fpm

    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fpm.h"', '#include "fpm_peak.h"',
             '#include "fpm_learn.h"', "int main(void) {"]
    for t, (cls, _) in STRUCTS.items():
        lines.append(f'printf("{t} size %zu\\n", sizeof({t}));')
        for f, _ in getattr(fpm, cls)._fields_:
            lines.append(f'printf("{t} {f} %zu\\n", offsetof({t}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    c_layout = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        t, f, v = line.split()
        c_layout[(t, f)] = int(v)
    for t, (cls, _) in STRUCTS.items():
        k = getattr(fpm, cls)
        assert ctypes.sizeof(k) == c_layout[(t, "size")], t
        for f, _ in k._fields_:
            assert getattr(k, f).offset == c_layout[(t, f)], (t, f)
