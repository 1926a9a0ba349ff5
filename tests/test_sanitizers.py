"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the host code
(CPU only; GPU code is not instrumented).

* The oracle: tests/sanitize/oracle_driver.c steps every flag of the oracle
  on small grids, in the sequential and the OpenMP build (gcc).
* The runtime: tests/sanitize/host_driver.c calls the host-only entry points
  of the C-ABI (defaults, derivation, every validation rule, EOS helpers,
  sizes, initial-density checks, null arguments) on a build of the library
  whose host code carries the sanitizers (hipcc, -Xarch_host); lbm_create
  and lbm_pool_create stop at their first device call when no GPU is
  present.  With a GPU the same driver also runs a simulation and a pool
  ("gpu" argument).
Any sanitizer report aborts the program, which fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1803_01756_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=timeout)
    return r.returncode, r.stdout


@pytest.mark.parametrize("omp", [False, True])
def test_oracle_under_sanitizers(tmp_path, omp):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    rc, out = _run(["gcc", "-O1", "-std=c11"] + SAN + (["-fopenmp"] if omp else []) +
                   ["-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm"])
    assert rc == 0, out
    env = dict(os.environ, OMP_NUM_THREADS="4")
    rc, out = _run([exe], env=env)
    print(out)
    assert rc == 0 and "0 non-finite" in out, out


def test_runtime_host_code_under_sanitizers(tmp_path):
    from sanitize.build import build_runtime_driver
    exe = build_runtime_driver(str(tmp_path))
    # the HIP runtime's own allocations are not ours to check for leaks
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    rc, out = _run([exe], env=env)
    print(out)
    assert rc == 0 and "0 failed expectations" in out, out
