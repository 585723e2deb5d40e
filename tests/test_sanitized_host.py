"""The library's host code (argument validation, error paths, context handling)
built with undefined-behaviour checks in trap mode (signed overflow, shifts, bounds,
null and misaligned access, invalid enum/bool loads, ...): the host checks of
test_library_host.py run against that build in a child process, where any check
that fires ends the process with SIGILL.  Device code is built as usual; no
sanitizer runtime is needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
UBSAN = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize-trap=undefined"]


@pytest.fixture(scope="module")
def sanitized_library(tmp_path_factory):
    sys.path.insert(0, ROOT)
    from paper_1709_09073_amd import build as B
    out = str(tmp_path_factory.mktemp("ubsan") / "librlbm.so")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")] + B.HIPCC_FLAGS + UBSAN + B.SOURCES + ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def test_host_checks_under_undefined_behaviour_traps(sanitized_library):
    env = dict(os.environ, RLBM_TEST_LIBRARY=sanitized_library)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_library_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-3000:], r.stderr[-2000:])
