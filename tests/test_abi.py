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
@pytest.mark.parametrize("header", ["fpm.h", "fpm_learn.h"])
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
    for n in fpm.EXPORTS + fpm.LEARN_EXPORTS:
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
