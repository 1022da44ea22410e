"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the HIP library is rebuilt with the sanitizers on its host pass only (the
device code is built as usual), and the host-side ABI tests run against it in a
child process with the sanitizer runtime preloaded: plan construction, option
and state checks, workspace sizing, the slab and undersampling tables, the
tuned-shape options and the batch argument checks, with no GPU."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang"
# each sanitizer flag goes to the host compilation only
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def _runtime():
    if not os.path.exists(CLANG):
        return None
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isfile(path) else None


@pytest.mark.timeout(900)
def test_host_abi_under_asan_and_ubsan(tmp_path):
    rt = _runtime()
    if rt is None:
        pytest.skip("no clang sanitizer runtime")
    sys.path.insert(0, os.path.join(ROOT, "paper_1910_06409_amd", "csrc"))
    try:
        import build as gke_build
    finally:
        sys.path.pop(0)
    lib = str(tmp_path / "libgke_san.so")
    gke_build.build(extra=SAN_FLAGS, lib=lib, obj_dir=str(tmp_path / "obj"))
    env = dict(os.environ, GKE_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in tail and "runtime error" not in tail
