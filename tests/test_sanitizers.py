"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The FP64 oracle (voge_oracle.c, built with clang without OpenMP) and the host
side of libvoge (argument checks, batch planning and workspace layout, built
with the sanitizers on the host pass only; the gfx950 code is unchanged) are
built out of tree with -fsanitize=address,undefined, and the oracle pins, the
noise-floor checks and the C-ABI tests run against them in a child process
with the sanitizer runtime preloaded.  Any report fails the run.  No GPU code
runs under a sanitizer.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-shared-libsan", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]


def _runtime():
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang is not installed")
def test_oracle_and_host_code_are_clean_under_asan_and_ubsan(tmp_path):
    rt = _runtime()
    assert rt, "clang's AddressSanitizer runtime is missing"
    oracle_so = str(tmp_path / "libvoge_oracle.so")
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared"] + SAN +
                   ["-o", oracle_so, os.path.join(ROOT, "oracle", "voge_oracle.c"), "-lm"], check=True)
    sys.path.insert(0, ROOT)
    from paper_2205_15401_amd import build as B
    host = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-shared-libsan"):
        host += ["-Xarch_host", f]
    lib_so = B.build(out=str(tmp_path / "libvoge.so"), extra=["-O1", "-g", "-fno-omit-frame-pointer"] + host,
                     link_extra=host)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", VOGE_ORACLE_LIB=oracle_so, VOGE_LIBRARY=lib_so)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_noise_floor.py"),
           os.path.join(ROOT, "tests", "test_abi.py")]
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=1500)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    for bad in ("AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert bad not in text, text[-4000:]
    assert " passed" in text
