"""The host side of the library (problem validation, workspace planning,
tiling choice, argument checks of every entry point) under AddressSanitizer:
the CPU tests of the C ABI rerun in a child process against
libjkcals_asan.so (api.cpp built with -fsanitize=address on its host side
only) with the clang ASan runtime preloaded.  Any invalid access or
use-after-free in that code aborts the child with an ASan report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2112_03985_amd", "libjkcals_asan.so")


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_abi_host_code_under_address_sanitizer():
    rt = _asan_runtime()
    if not os.path.exists(LIB) or rt is None:
        pytest.skip("host-sanitizer build or the clang ASan runtime not present "
                    "(python -m paper_2112_03985_amd.build builds the former)")
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "JKCALS_LIBRARY": LIB,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1"})
    code = ("import sys, pytest, paper_2112_03985_amd as jk\n"
            "jk.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "assert 'libjkcals_asan.so' in maps and 'libclang_rt.asan' in maps\n"
            "sys.exit(pytest.main(['-q', '-m', 'not gpu', '-p', 'no:cacheprovider', "
            "'tests/test_abi.py', 'tests/test_split_layout.py']))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr
