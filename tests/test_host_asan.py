"""The library's host code (runtime argument checks, the KD-tree crop, status
strings, configuration) under AddressSanitizer: tests/test_abi.py is run in a
child process against libgsr_asan.so (host passes instrumented) with the clang
ASan runtime preloaded. No GPU is used."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_lib():
    from paper_2403_11367_amd import build
    srcs = glob.glob(os.path.join(build.CSRC, "*"))
    if not os.path.exists(build.LIB_ASAN) or os.path.getmtime(build.LIB_ASAN) < max(map(os.path.getmtime, srcs)):
        build.build(asan=True)
    return build.LIB_ASAN, build.asan_runtime()


def test_abi_tests_pass_under_asan():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only run; a GPU is present")
    lib, rt = _asan_lib()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", GSR_LIB=lib)
    probe = ("import paper_2403_11367_amd.gsr as g; m = open('/proc/self/maps').read(); "
             "assert 'libgsr_asan.so' in m and 'libclang_rt.asan' in m, 'ASan build not loaded'; print('ok')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr
