"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU.

Every source is compiled for the host only (hipcc --cuda-host-only: kernels become launch
stubs, no device code is built), instrumented with both sanitizers, and linked with
tests/host_sanitize/driver.cpp, which fills in a context by hand and calls the host-side setup
(primitive polynomials, Sobol' matrices), every entry point's argument validation with invalid
arguments, the workspace sizes and the tuning-file reader on malformed files.  A sanitizer
report aborts the run; the setup outputs are compared with the oracle.  The device fat binaries
the host objects refer to are replaced by empty stand-ins (nothing is launched).
"""

import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import digital

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_15584_amd", "csrc")
SOURCES = ["context.hip", "setup.cpp", "generate.hip", "integrate.hip", "tune.hip"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        pytest.skip("hipcc not available")
    return h


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    hipcc = _hipcc()
    d = tmp_path_factory.mktemp("host_san")
    common = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"),
              "-I", CSRC] + SAN
    objs = []
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp")]
    procs = []
    for src in srcs:
        obj = str(d / (os.path.basename(src) + ".o"))
        procs.append((src, subprocess.Popen([hipcc] + common + ["-c", src, "-o", obj], stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, "compiling %s failed:\n%s" % (src, out)
    # empty stand-ins for the device fat binaries the host objects refer to
    nm = subprocess.run(["nm", "-u"] + objs, capture_output=True, text=True, check=True).stdout
    syms = sorted(set(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", nm)))
    stub = d / "fatbin_stub.cpp"
    stub.write_text("".join('extern "C" __attribute__((used)) const unsigned char %s[64] = {0};\n' % s for s in syms))
    subprocess.run(["g++", "-c", str(stub), "-o", str(d / "fatbin_stub.o")], check=True)
    exe = str(d / "driver")
    link = subprocess.run([hipcc] + SAN + objs + [str(d / "fatbin_stub.o"), "-o", exe], capture_output=True, text=True)
    assert link.returncode == 0, link.stdout + link.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe, str(d)], capture_output=True, text=True, env=env, timeout=300)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]
    return r.stdout


def _values(out, key):
    line = next(l for l in out.splitlines() if l.startswith(key + ":"))
    return np.array([int(v) for v in line.split(":", 1)[1].split()], dtype=np.uint64)


def test_no_sanitizer_reports_and_every_status_as_expected(driver_output):
    assert "failures 0" in driver_output
    assert "MISMATCH" not in driver_output


def test_setup_outputs_equal_the_oracle(driver_output):
    from oracle.digital import primitive_polynomials

    assert list(_values(driver_output, "poly")) == primitive_polynomials(300)
    for s in (1, 7, 64):
        di = np.zeros((s, 16), dtype=np.uint64)
        for j in range(s):
            for k in range(16):
                v = ((j * 16 + k) * 2654435761) & 0xFFFFFFFF
                di[j, k] = (v | 1) & ((2 << k) - 1)
        want = digital.sobol_matrices(s, di.astype(np.uint32))
        assert np.array_equal(_values(driver_output, "mats_%d" % s).reshape(s, 32), want)
        wide = _values(driver_output, "wide_%d" % s).reshape(s, 64)
        assert np.array_equal(wide[:, :32], want)


def test_workspace_sizes(driver_output):
    sizes = dict(re.findall(r"^(ws_\w+_bytes) (\d+)$", driver_output, flags=re.M))
    assert int(sizes["ws_lobes_bwd_bytes"]) == 1024 + 640 * 64 * 17
    assert int(sizes["ws_lobes_step_bytes"]) == 1024 + 640 * (64 * 17 + 1)
    # Genz: the pixel list (4 B per pixel) and 90 bucket counts per 1024 pixels, beside the task
    # counters, the Sobol' tables and the bucket totals
    P = 1920 * 1080
    lo = 4 * P + 90 * 4 * -(-P // 1024)
    assert lo <= int(sizes["ws_genz_bytes"]) <= lo + 8192
