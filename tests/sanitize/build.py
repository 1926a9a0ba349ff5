"""Builds of the host-side sanitizer drivers (test infrastructure).

build_runtime_driver(out_dir): the library with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code only (-Xarch_host; the GPU code
is not instrumented) and host_driver.c linked against it; returns the
driver's path.  The default out_dir is tests/sanitize/_build, where
__graft_entry__.build() puts it so that the GPU test can run it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1803_01756_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]
DEFAULT_DIR = os.path.join(HERE, "_build")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), r.stdout))


def build_runtime_driver(out_dir: str = DEFAULT_DIR) -> str:
    import sys
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1803_01756_amd import build as B
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "liblbm_san.so")
    srcs = [os.path.join(CSRC, s) for s in B.SOURCES if os.path.exists(os.path.join(CSRC, s))]
    host_san = []
    for f in SAN[:-1]:
        host_san += ["-Xarch_host", f]
    _run([B.hipcc(), "--offload-arch=" + B.ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
          "-mcode-object-version=5", "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-g"] + host_san +
         ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", lib] + srcs)
    exe = os.path.join(out_dir, "host_driver")
    _run([B.hipcc(), "-x", "c", "-O1"] + SAN + ["-I", os.path.join(ROOT, "include"), "-o", exe,
         os.path.join(HERE, "host_driver.c"), "-L", out_dir, "-llbm_san", "-Wl,-rpath," + out_dir,
         "-lm"])
    return exe
