"""Host code under the address and undefined-behaviour sanitizers.

The oracle (every entry point on a ragged random case) is rebuilt here with
gcc's sanitizers and run; the library's host API, built with host-only
instrumentation by tests/sanitize/build.py (part of the build entry point),
runs its argument checks without a device and, under the gpu marker, a short
session on device 0 (re-binning, both dtypes, fused null collisions,
replays, the allocation-free form, the variants, a workspace cap and an
injected NaN).  Any report aborts the driver with a non-zero status."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "sanitize"))
import build as san  # noqa: E402  (tests/sanitize/build.py)


def _run(cmd, leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={int(leaks)}:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, f"{cmd} -> {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


def test_oracle_under_sanitizers():
    exe = san.build_oracle_driver()
    assert "oracle driver ok" in _run([exe], leaks=True)


def _api_driver():
    exe = san.API_DRIVER
    src = [os.path.join(HERE, "sanitize", "api_driver.cpp")]
    stale = not os.path.exists(exe) or any(os.path.getmtime(s) > os.path.getmtime(exe) for s in src)
    return exe, stale


def test_api_argument_checks_under_sanitizers():
    exe, stale = _api_driver()
    if stale:
        exe = san.build_api_driver()
    assert "api driver ok" in _run([exe], leaks=True)


@pytest.mark.gpu
def test_api_device_session_under_sanitizers():
    exe, stale = _api_driver()
    assert not stale, "sanitised API driver missing or older than its source: run the build"
    # the HIP runtime keeps allocations until exit: leak checking stays off here
    assert "api driver ok" in _run([exe, "--device"], leaks=False)
