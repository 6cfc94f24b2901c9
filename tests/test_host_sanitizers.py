"""The C-ABI CPU tests run against the library built with its host code under AddressSanitizer
and UndefinedBehaviorSanitizer (build.build_sanitized: plan, runtime and host math, linked with
the normal kernel objects; device code is never sanitized), in a child interpreter with the
sanitizer runtime preloaded.  A second child writes past the end of an output array through
pkm_wedges, to show that the instrumentation is live: the sanitizer must stop it."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def san_env():
    from paper_1704_02357_amd import build as b
    if not all(os.path.exists(os.path.join(b.BUILD, k)) for k in ("kernels_paint.o", "kernels_fft.o")):
        b.build()
    lib = b.build_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=b.sanitizer_runtime(), PKM_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    return env


def test_capi_tests_pass_under_sanitizers(san_env):
    check = ("from paper_1704_02357_amd.pkm import lib_path, load_library; "
             "import ctypes; lib = load_library(); "
             "assert lib_path().endswith('libpkm_san.so'); "
             "ctypes.CDLL(lib_path()).__asan_report_load8; print('sanitized library loaded')")
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=san_env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_capi_cpu.py", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=san_env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_sanitizer_catches_an_overrun(san_env):
    code = ("import ctypes as C, numpy as np; from paper_1704_02357_amd.pkm import load_library; "
            "lib = load_library(); P = lambda a: a.ctypes.data_as(C.c_void_p); "
            "poles = np.ones((3, 64)); mu = np.linspace(0.0, 1.0, 4); out = np.empty(8); "
            "lib.pkm_wedges(P(poles), 4, 64, P(mu), 4, P(out))")  # needs 64 x 3 outputs
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san_env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, (r.returncode, r.stderr[-2000:])
