"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: the library is
rebuilt with both on its host side (device code unchanged) and the host-only ABI tests (layout
queries, argument validation, defaults, the lifecycle and map refusals) run against it in a
child process with the sanitizer runtime preloaded; any report fails the test.  No GPU call."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_only_abi_tests_pass_under_address_and_undefined_behaviour_sanitizers():
    from paper_2510_26358_amd import build
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("the ROCm compiler is not available")
    lib = build.build(verbose=False, sanitize=True)
    rt = build.sanitizer_runtime()
    # the runtime must come first among the preloaded libraries; anything already preloaded stays
    preload = ":".join(p for p in (rt, os.environ.get("LD_PRELOAD", "")) if p)
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", AGS_LIBRARY=lib)
    code = ("import ctypes, sys, pytest\n"
            "assert hasattr(ctypes.CDLL(None), '__asan_init')  # the runtime is live\n"
            "from paper_2510_26358_amd import _lib\n"
            "assert _lib.LIB_PATH.endswith('libagsplat_san.so'), _lib.LIB_PATH\n"
            "rc = pytest.main(['-q', '-p', 'no:cacheprovider', 'tests/test_abi.py'])\n"
            "assert _lib._lib is not None and _lib._lib._name.endswith('libagsplat_san.so')\n"
            "sys.exit(int(rc))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out, out[-2000:]
