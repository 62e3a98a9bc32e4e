"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (tests/host_sanitize): a C driver calls the C ABI through
validation and error paths on the CPU, and through whole context, filter and
batch lifecycles (graph capture, re-capture after tile changes, restart,
tuning) on the GPU.  Any sanitizer finding or unexpected status fails."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "host_sanitize"))
import build as sanbuild  # noqa: E402

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _stale():
    if not os.path.exists(sanbuild.DRIVER):
        return True
    t = os.path.getmtime(sanbuild.DRIVER)
    srcs = [os.path.join(sanbuild.CSRC, f) for f in os.listdir(sanbuild.CSRC)]
    srcs += [os.path.join(HERE, "host_sanitize", "driver.cpp"),
             os.path.join(os.path.dirname(HERE), "include", "atns.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


def _run(mode, timeout):
    r = subprocess.run([sanbuild.DRIVER, mode], capture_output=True, text=True, env=ENV, timeout=timeout)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0 and "driver ok" in r.stdout, out[-4000:]


def test_host_code_under_sanitizers_cpu():
    if _stale():
        sanbuild.build()
    _run("cpu", 120)


@pytest.mark.gpu
def test_host_code_under_sanitizers_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(sanbuild.DRIVER), "sanitizer driver not built (__graft_entry__.build())"
    print("[case] sanitized host lifecycle on the GPU", flush=True)
    _run("gpu", 240)
