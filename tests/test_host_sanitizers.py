"""The host C++ of the library (the multithreaded host indexing and the
argument checks of the C ABI) built with AddressSanitizer +
UndefinedBehaviorSanitizer and, separately, with ThreadSanitizer, and run on
seeded problems: no sanitizer report, and the indexing counts equal the
oracle's.  CPU only: the driver (tests/sanitize/host_indexing_driver.cpp)
calls cb_host_indexing repeatedly (the worker pool is reused across calls)
and one cb_setup that validation rejects before any device work.  The
device objects are linked unchanged from the library build."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import assemble, topology

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_06323_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
DEVICE_OBJS = [os.path.join(BUILD, f + ".hip.o") for f in ("integrate", "indexing", "operator", "dense", "bddc",
                                                            "nitsche", "manufactured", "coarse_nd")]
GXX = shutil.which("g++")

pytestmark = pytest.mark.skipif(
    GXX is None or not all(os.path.exists(o) for o in DEVICE_OBJS) or not os.path.exists("/opt/rocm/lib"),
    reason="needs g++, the ROCm runtime and the library's device objects (paper_1703_06323_amd.build)")

SANITIZERS = {
    "address_undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "thread": ["-fsanitize=thread"],
}


def _cases():
    out = [W.single_ball(), W.single_ball().with_options(coarse_variant=0), W.random_balls(16, 4, 6, 3),
           W.random_balls(24, 8, 10, 4).with_options(objects=1), W.random_balls(32, 8, 14, 5),
           W.random_balls(20, 4, 30, 8), W.uncut(12, 4), W.random_balls(8, 8, 3, 5)]
    rng = np.random.default_rng(17)
    for k in range(4):
        n, s = [(12, 3), (16, 4), (10, 5), (24, 8)][k]
        out.append(W.random_balls(n, s, int(rng.integers(5, 30)), 300 + k).with_options(
            coarse_variant=int(rng.integers(0, 2))))
    return out


def _write_cases(path, probs):
    expect = []
    with open(path, "wb") as fh:
        fh.write(struct.pack("i", len(probs)))
        for p in probs:
            d = assemble.discretise(p)
            t = topology.build(p, d)
            fh.write(struct.pack("iiiii", p.n, p.s, p.n_balls, p.coarse_variant, p.objects))
            fh.write(np.ascontiguousarray(p.centres, dtype=np.float64).tobytes())
            fh.write(np.ascontiguousarray(p.radii, dtype=np.float64).tobytes())
            fh.write(np.ascontiguousarray(d.count, dtype=np.int32).tobytes())
            expect.append(f"{d.dof_node.size} {t.n_coarse} {t.obj_type.size} {t.obj_dofs.size}")
    return expect


def _build(tmp, flags):
    common = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-pthread", *flags]
    srcs = [(os.path.join(CSRC, "cutbddc.cpp"), ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                                 "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]),
            (os.path.join(CSRC, "topology.cpp"), ["-I" + CSRC]),
            (os.path.join(ROOT, "tests", "sanitize", "host_indexing_driver.cpp"), ["-I" + os.path.join(ROOT, "include")])]
    procs, objs = [], []
    for src, inc in srcs:
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([GXX, "-c", *common, *inc, src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    exe = os.path.join(tmp, "driver")
    r = subprocess.run([GXX, *flags, "-pthread", *objs, *DEVICE_OBJS, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


@pytest.mark.parametrize("kind", list(SANITIZERS))
def test_host_code_sanitizer_clean(kind, tmp_path):
    cases = str(tmp_path / "cases.bin")
    expect = _write_cases(cases, _cases())
    exe = _build(str(tmp_path), SANITIZERS[kind])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=0")
    r = subprocess.run([exe, cases, "3"], capture_output=True, text=True, env=env, timeout=600)
    report = r.stderr
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "WARNING: ThreadSanitizer" not in report, report[-4000:]
    assert r.returncode == 0, (r.returncode, report[-4000:])
    lines = r.stdout.split("\n")
    assert lines[:len(expect)] == expect
    assert lines[len(expect)] == "setup_error -1"
