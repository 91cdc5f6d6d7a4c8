"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the oracle (g++) and the host emulation of the device arithmetic (hipcc,
host pass only), each driven over every routine on small grids.  Any invalid
access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def run(exe, tmp_path):
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok"), r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_oracle")
    src = [os.path.join(ROOT, "oracle", "pclb_oracle.cpp"), os.path.join(NATIVE, "sanitize_oracle.cpp")]
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                    "-fno-omit-frame-pointer", *SAN, "-o", exe, *src], check=True)
    run(exe, tmp_path)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_device_math_emulation_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_emulate")
    host_san = [x for s in SAN for x in ("-Xarch_host", s)]
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "-ffp-contract=on",
                    "-fno-omit-frame-pointer", *host_san, "-x", "hip", "--cuda-host-only",
                    "-o", exe, os.path.join(NATIVE, "sanitize_emulate.cpp")], check=True)
    run(exe, tmp_path)
