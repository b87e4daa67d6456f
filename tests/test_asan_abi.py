"""The library's host code under AddressSanitizer: tests/asan/build.sh
builds libmpofit with -fsanitize=address on the host pass only (device code
as usual) and a C driver that exercises the C ABI's host-side paths
(workspace queries, validation, error strings); the driver must report no
failure and ASan no error.  No device is touched.  The build (about two
minutes) is cached per source hash under the system temp directory."""
import hashlib
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hash():
    h = hashlib.sha1()
    for rel in ["tests/asan/build.sh", "tests/asan/abi_driver.c", "include/mpofit.h"] + [
            f"paper_2606_23274_amd/csrc/{f}" for f in sorted(os.listdir(os.path.join(ROOT, "paper_2606_23274_amd/csrc")))]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_host_abi_under_address_sanitizer():
    out = os.path.join(tempfile.gettempdir(), f"mpofit_asan_{_hash()}")
    driver = os.path.join(out, "abi_driver")
    if not os.path.exists(driver):  # (the driver is linked last: it marks a complete build)
        shutil.rmtree(out, ignore_errors=True)
        r = subprocess.run(["bash", os.path.join(ROOT, "tests/asan/build.sh"), out], capture_output=True,
                           text=True, timeout=1200)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([driver], capture_output=True, text=True, timeout=300, env=env, cwd=tempfile.gettempdir())
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
