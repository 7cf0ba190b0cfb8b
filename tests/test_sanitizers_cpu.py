"""The FP64 oracle and the host side of the library built and run under
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the device
code of the library is built normally).  The oracle driver runs small
lattices through every code path of the oracle; the library driver calls
the host-side paths of the C ABI that need no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "oracle"),
                           os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "dmrt_oracle.c"), "-lm", "-o", exe])
    out = _run(exe)
    assert out.count("bad 0") == 5, out


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1503_08406_amd", "csrc")
    srcs = sorted(os.path.join(csrc, n) for n in os.listdir(csrc) if n.endswith(".hip"))
    exe = str(tmp_path / "abi_san")
    # sanitizers for the host pass only: each flag behind -Xarch_host
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
                           "-I", os.path.join(ROOT, "include"), "-x", "hip", *srcs, "-x", "c++",
                           os.path.join(HERE, "sanitize", "abi_driver.c"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    assert "host ABI paths ok" in _run(exe)
