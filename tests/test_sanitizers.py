"""The oracle and the library's host-side logic under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only; no device code runs).

* `sanitize/oracle_driver.c` runs the oracle's entry points (init, steps,
  float mesh decision, frozen step, counts, mass, adjoint primitives) on small
  cases of every scheme, gamma, metric and wall kind, built with gcc.
* `sanitize/host_driver.hip` includes the library source and runs its
  parameter checks and plans over a sweep of valid and invalid sets, the
  transport tables of every scheme, gamma and wall case, and the tree checks
  on hand-built trees; the sanitizers instrument the host code only.

A sanitizer finding aborts the driver (no recovery), which fails the test.
The builds are cached by a hash of their sources.
"""
import hashlib
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
BUILD = os.path.join(SAN, "_build")
CSRC = os.path.join(ROOT, "paper_2103_02903_amd", "csrc")


def _digest(paths, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _build(name, sources, cmd):
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "%s_%s" % (name, _digest(sources, cmd)))
    if not os.path.exists(out):
        tmp = out + ".tmp"
        res = subprocess.run(cmd + ["-o", tmp], capture_output=True, text=True)
        assert res.returncode == 0, res.stdout + res.stderr
        os.replace(tmp, out)
    return out


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    return res.stdout


def test_oracle_under_sanitizers():
    srcs = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "mr_oracle.c"),
            os.path.join(ROOT, "oracle", "mr_oracle.h")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
           srcs[0], srcs[1], "-lm"]
    out = _run(_build("oracle_driver", srcs, cmd))
    assert out.count("mass") == 9


@pytest.mark.timeout(900)
def test_library_host_logic_under_sanitizers():
    srcs = [os.path.join(SAN, "host_driver.hip"), os.path.join(ROOT, "include", "mrlbm.h")] + \
        [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".h"))]
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    # sanitizers on the host code only (the device code is built plain and never runs)
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wno-c++20-extensions", "-I", os.path.join(ROOT, "include"), srcs[0]]
    out = _run(_build("host_driver", srcs, cmd))
    assert "host checks passed" in out
