"""AddressSanitizer / UndefinedBehaviorSanitizer run of the host code (CPU):
the oracle through every entry point, and the library's host translation units
under the host C-ABI tests (tests/sanitize/run_host_asan.sh).  Needs the kernel
objects of a prior build (paper_2010_15595_amd/_build)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2010_15595_amd", "_build")


@pytest.mark.slow
def test_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(os.path.join(BUILD, "lhaf_kernels.hip.o")) or not shutil.which("gcc"):
        pytest.skip("needs a prior library build and gcc")
    env = {k: v for k, v in os.environ.items() if k not in ("LD_PRELOAD", "GBS_LIB_PATH")}
    r = subprocess.run(["bash", os.path.join(ROOT, "tests", "sanitize", "run_host_asan.sh"), str(tmp_path)],
                       capture_output=True, text=True, env=env, timeout=900)
    tail = "\n".join((r.stdout + r.stderr).splitlines()[-30:])
    assert r.returncode == 0, tail
    assert "host sanitizer run clean" in r.stdout
    assert "runtime error" not in r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stdout + r.stderr
