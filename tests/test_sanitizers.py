"""Address and undefined-behaviour sanitizer builds (CPU): the oracle with
its entry points driven on small inputs (tests/sanitize/oracle_main.cpp),
and the library's host-only code -- mesh validation and the breadth-first
tree build, line quantities -- compiled with the sanitizers on the host
side only (tests/sanitize/host_main.cpp; no device is touched).  Any
report aborts the driver, which the test sees as a failure."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _run(cmd, cwd):
    p = subprocess.run(cmd, cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert p.returncode == 0, " ".join(cmd) + "\n" + p.stdout[-4000:]
    return p.stdout


def _host_san():
    # each sanitizer flag applies to the host compilation only
    out = []
    for f in SAN_FLAGS:
        out += ["-Xarch_host", f]
    return out


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-ffp-contract=off", "-fno-omit-frame-pointer"] + SAN_FLAGS +
         ["-I" + os.path.join(ROOT, "oracle"), "-o", exe, os.path.join(SAN, "oracle_main.cpp"),
          os.path.join(ROOT, "oracle", "oracle.cpp")], str(tmp_path))
    out = _run([exe], str(tmp_path))
    assert "0 failures" in out


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_code_under_sanitizers(tmp_path):
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2001_11252_amd", "csrc")]
    csrc = os.path.join(ROOT, "paper_2001_11252_amd", "csrc")
    t = str(tmp_path)
    # kernels as built for the library (their host part is launch glue)
    _run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"] + inc + ["-c", os.path.join(csrc, "rmc_kernels.hip"), "-o", "k.o"], t)
    for src, obj in ((os.path.join(csrc, "rmc_api.cpp"), "api.o"), (os.path.join(SAN, "host_main.cpp"), "main.o")):
        _run([HIPCC, "--offload-arch=gfx950", "--offload-host-only", "-O1", "-g", "-std=c++17",
              "-fno-omit-frame-pointer"] + _host_san() + inc + ["-c", src, "-o", obj], t)
    _run([HIPCC, "--offload-arch=gfx950"] + _host_san() + ["-o", "host_san", "main.o", "api.o", "k.o"], t)
    out = _run([os.path.join(t, "host_san")], t)
    assert "0 failures" in out
