"""Host sanitizer builds of the CPU oracle (CPU only).

``oracle/oracle.c`` is compiled with the driver ``tests/sanitize/oracle_sanitize.c``
under AddressSanitizer + UndefinedBehaviorSanitizer (leak checking on, every
report fatal) and, separately, under ThreadSanitizer, which watches the
threaded brute-force matcher.  The driver calls every exported oracle function
on seeded synthetic inputs (empty and 255-byte strings, bytes outside the
symbol map, empty dictionaries and query sets, every fingerprint variant at 16
and 32 bits, the error paths) and checks properties the mathematics fixes
(distance axioms, Eq. 1 soundness, brute-force counts).  Before trusting a
clean run, each sanitizer must report a planted fault in a small probe
program, so that a pass is not the result of a runtime that never started."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_sanitize.c")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=thread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", TSAN_OPTIONS="halt_on_error=1:exitcode=25")

PROBES = {  # planted fault each sanitizer must report, built with that sanitizer alone
    "address": ("#include <stdlib.h>\nint main(void){ volatile char *p = malloc(8); p[8] = 1; free((void*)p); return 0; }\n",
             "heap-buffer-overflow"),
    "undefined": ("#include <limits.h>\nint main(int c, char **v){ (void)v; int x = INT_MAX - 1 + c; x += c; return x & 1; }\n",
              "signed integer overflow"),
    "thread": ("#include <pthread.h>\nvolatile int x;\n"
               "void *f(void *a){ (void)a; for (int i = 0; i < 100000; ++i) x++; return 0; }\n"
               "int main(void){ pthread_t t; pthread_create(&t, 0, f, 0); for (int i = 0; i < 100000; ++i) x++;\n"
               "  pthread_join(t, 0); return 0; }\n",
             "data race"),
}


def _compile(tmp_path, name, sources, flags):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-Wall", "-Wextra", "-Werror", "-pthread", *flags, *sources, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    return exe if r.returncode == 0 else None, r.stderr


def _probe(tmp_path, kind):
    src, report = PROBES[kind]
    flags = [f"-fsanitize={kind}"]
    path = tmp_path / f"probe_{kind}.c"
    path.write_text(src)
    exe, err = _compile(tmp_path, f"probe_{kind}", [str(path)], flags)
    if exe is None:
        pytest.skip(f"gcc cannot build with {flags[0]} here: {err.strip()[:200]}")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=ENV)
    if "FATAL" in r.stderr and report not in r.stderr:
        pytest.skip(f"{kind} runtime does not start here: {r.stderr.strip()[:200]}")
    assert r.returncode != 0 and report in r.stderr, (kind, r.returncode, r.stderr[-2000:])


@pytest.fixture(scope="module", autouse=True)
def _gcc():
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")


def test_asan_ubsan_build_of_the_oracle_is_clean(tmp_path):
    _probe(tmp_path, "address")
    _probe(tmp_path, "undefined")
    exe, err = _compile(tmp_path, "oracle_asan", [ORACLE, DRIVER], ASAN)
    assert exe, err
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR:" not in r.stderr, r.stderr[-4000:]
    assert "all checks passed" in r.stdout


def test_tsan_build_of_the_threaded_matcher_is_clean(tmp_path):
    _probe(tmp_path, "thread")
    exe, err = _compile(tmp_path, "oracle_tsan", [ORACLE, DRIVER], TSAN)
    assert exe, err
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
