"""The runtime's host code under AddressSanitizer and UndefinedBehaviorSanitizer
with the GPU: tests/sanitize/host_driver.c in its "gpu" mode (a simulation
in every storage and several options, a pool under a binding cap, and 400
random pool operations), linked against the library built with sanitizers
on its host code only.  __graft_entry__.build() builds it into
tests/sanitize/_build; any sanitizer report or failed expectation fails the
test."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "_build", "host_driver")


def test_host_code_with_gpu_under_sanitizers():
    print("\n[case] sanitized host driver, gpu mode", flush=True)
    assert os.path.exists(EXE), "the sanitized driver is built by __graft_entry__.build()"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    r = subprocess.run([EXE, "gpu"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=240)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0 and "0 failed expectations" in r.stdout
