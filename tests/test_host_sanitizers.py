"""The host-only parts of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU): the kernel basis on its exact path
(Hermite form + exact LLL) and on its reduction-interleaved path (the iid
sparse law), and the inequality lift, built with g++ from the library's own
sources together with tests/host_sanitize/driver.cpp.  The sanitized build
must report nothing and return the regular library's results bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2412_13576_amd import graver as G
from paper_2412_13576_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_13576_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("asan") / "driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"), os.path.join(CSRC, "lattice.cpp"),
           os.path.join(CSRC, "inequality.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _ints(a):
    return " ".join(str(int(x)) for x in np.asarray(a).ravel())


def test_host_library_under_sanitizers(driver, tmp_path):
    insts = [(W.tiny_instance(1000).A, 1), (W.tiny_instance(1003).A, 0), (W.random_instance(7, 3, 9).A, 1),
             (W.qp_instance(2000).A, 1), (W.sparse_quadratic_instance(4150, 150, 45).A, 1)]
    lifts = []
    tiny = W.tiny_instance(1001)
    Gm, h = W.inequality_rows(tiny, 3, seed=5)
    lifts.append((tiny, Gm, h))
    with open(tmp_path / "in.txt", "w") as fh:
        for A, lll in insts:
            fh.write(f"basis {A.shape[0]} {A.shape[1]} {lll} {_ints(A)}\n")
        for inst, Gm, h in lifts:
            fh.write(f"lift {inst.A.shape[0]} {inst.n} {Gm.shape[0]} {_ints(inst.A)} {_ints(inst.b)} {_ints(inst.l)} "
                     f"{_ints(inst.u)} {_ints(Gm)} {_ints(h)}\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, str(tmp_path / "in.txt"), str(tmp_path / "out.txt")], capture_output=True,
                       text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    lines = open(tmp_path / "out.txt").read().splitlines()
    assert len(lines) == len(insts) + len(lifts)
    for (A, lll), line in zip(insts, lines):
        w = line.split()
        assert w[0] == "basis" and int(w[1]) == 0
        d, n = int(w[2]), A.shape[1]
        Bs = np.array([int(x) for x in w[3:3 + n * d]], np.int64).reshape(n, d)
        Ps = np.array([float(x) for x in w[3 + n * d:]], np.float64).reshape(d, n)
        B, P = G.kernel_basis(A, lll=bool(lll))
        assert np.array_equal(Bs, B)
        assert np.array_equal(Ps.view(np.uint64), P.view(np.uint64))
    for (inst, Gm, h), line in zip(lifts, lines[len(insts):]):
        w = line.split()
        assert w[0] == "lift" and int(w[1]) == 0
        A2, b2, l2, u2, _ = G.lift_inequalities(inst.A, inst.b, inst.l, inst.u, Gm, h)
        expect = np.concatenate([A2.ravel(), b2, l2, u2]).astype(np.int64)
        assert np.array_equal(np.array([int(x) for x in w[2:]], np.int64), expect)
