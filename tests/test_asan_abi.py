"""Host AddressSanitizer run of the C ABI.

tests/asan/abi_driver.cpp calls the library through include/nssdoa.h the way a user does (argument
checks, error paths, every estimator, graph capture, the streaming pipeline, the network), linked
against libnssdoa_asan.so: the library with its host code instrumented by AddressSanitizer
(paper_2007_14135_amd.build.build_asan).  A run passes when every call returns what it should and
ASan reports no invalid access and LeakSanitizer no leak of the library's allocations
(tests/asan/lsan.supp lists the ROCm runtime's own, which live until the process ends).
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "asan", "_build", "abi_driver")
SUPP = os.path.join(ROOT, "tests", "asan", "lsan.supp")


def _run(mode, timeout):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:exitcode=23"
    env["LSAN_OPTIONS"] = "suppressions=" + SUPP
    print("abi_driver", mode, flush=True)
    r = subprocess.run([DRIVER, mode], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, (r.returncode, out[-4000:])
    assert "0 failed checks" in out, out[-4000:]


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present: the device test covers these calls")
def test_host_asan_abi_without_device():
    if not os.path.exists(DRIVER):
        from paper_2007_14135_amd.build import build_asan
        build_asan()
    _run("cpu", 120)


@pytest.mark.gpu
def test_host_asan_abi_on_device():
    if not os.path.exists(DRIVER):
        pytest.skip("host-ASan driver not built (paper_2007_14135_amd.build.build_asan)")
    _run("gpu", 300)
