"""The oracle's C code built with AddressSanitizer and
UndefinedBehaviorSanitizer (every report aborts): every entry point is
called on small inputs in a child process, which must exit cleanly and give
the same results as the normal build."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _asan_runtime():
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_ubsan(tmp_path):
    import oracle

    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    ref = tmp_path / "plain.npz"
    san = tmp_path / "san.npz"
    env = dict(os.environ, OBEM_ORACLE_LIB=so, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_exercise.py"), str(san)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    sys.path.insert(0, HERE)
    import oracle_exercise

    oracle_exercise.run(str(ref))
    a, b = np.load(ref), np.load(san)
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        if a[k].dtype.kind in "iub":
            assert np.array_equal(a[k], b[k]), k
        else:
            np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=0, err_msg=k)
