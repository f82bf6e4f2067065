"""Host code of libnisqtol under AddressSanitizer and UndefinedBehaviorSanitizer.

The host sources (circuit loading, text format, planner, engine, C ABI,
surrogate host code) are compiled with both sanitizers on their host pass
(the device code is built as usual, without them), linked into a driver
program (tests/host_sanitize/driver.cpp) that exercises the host-only calls
and the error paths of the ABI on generated circuits, and run; any sanitizer
report fails the test.  No GPU is used: without one, nt_create must fail
cleanly.
"""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_07264_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SOURCES = ["circuit.cpp", "plan.cpp", "engine.cpp", "gnn_model.cpp", "capi.cpp"]
DEVICE_SOURCES = ["kernels.hip", "gnn.hip"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, (" ".join(cmd)) + "\n" + r.stdout + r.stderr
    return r


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = tmp_path_factory.mktemp("san")
    inc = ["-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = []
    for src in HOST_SOURCES:
        o = str(out / (src + ".o"))
        _run([HIPCC] + inc + SAN + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    dev_flags = ["--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-mllvm", "-simplifycfg-sink-common=false"]
    for src in DEVICE_SOURCES:
        o = str(out / (src + ".o"))
        _run([HIPCC] + inc + dev_flags + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    d = str(out / "driver.o")
    _run([HIPCC] + inc + SAN + ["-c", os.path.join(HERE, "driver.cpp"), "-o", d])
    exe = str(out / "driver")
    _run([HIPCC, "--offload-arch=gfx950", "-fno-gpu-sanitize", "-fsanitize=address", "-fsanitize=undefined",
          "-o", exe, d] + objs)
    return exe


def test_host_code_under_sanitizers(driver, tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("runs where no GPU is present (nt_create must fail)")
    rng = np.random.default_rng(4)
    circs = [W.config0(), W.config1(n=14, layers=6), W.config4(n=16, rounds=2), W.config2(2),
             W.quantum_volume(5, 4, rng), W.qft(9), W.ghz(3), W.Circuit(1, [W.Gate("H", (0,))])]
    paths = []
    for i, c in enumerate(circs):
        p = str(tmp_path / f"c{i}.txt")
        W.write_text(c, p)
        paths.append(p)
    env = dict(os.environ)
    # leaks are checked too; only the HIP runtime's own allocations, which
    # live until the process ends, are suppressed
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(HERE, "lsan.supp")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver] + paths, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "all checks passed" in r.stdout
