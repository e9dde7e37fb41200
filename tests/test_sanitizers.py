"""Host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two host-side codes are rebuilt with g++ and the sanitizers, then exercised in
a child process that preloads the ASan runtime (Python itself is not
instrumented, so leak checking is off):

- the FP64 oracle (oracle/oracle.cpp), driven by the whole oracle pin suite;
- the exact-predicate Delaunay triangulation of the point-cloud densification
  (csrc/delaunay.cpp), on random point sets, integer grids full of cocircular
  quadruples, and the inputs it must reject.

Any sanitizer report aborts the child, which fails the test.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GXX = shutil.which("g++")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

pytestmark = pytest.mark.skipif(GXX is None, reason="g++ is not installed")


def _asan_runtime():
    p = subprocess.run([GXX, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _env(**extra):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("the ASan runtime of g++ was not found")
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT, **extra)
    return env


def _build(out, sources, extra=()):
    cmd = [GXX, "-O2", "-std=c++17", "-fPIC", "-shared", *SAN, *extra, "-o", out, *sources]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _build(lib, [os.path.join(ROOT, "oracle", "oracle.cpp")], ["-fopenmp"])
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x",
                        "-q", "-p", "no:cacheprovider"], cwd=ROOT, env=_env(GS_ORACLE_LIB=lib),
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert " passed" in r.stdout


_DELAUNAY_STUB = """
#include <string>
#include "gs.h"
namespace gs {
gs_status fail(gs_status s, const std::string&) { return s; }
}
"""

_DELAUNAY_DRIVER = textwrap.dedent("""
    import ctypes as C, sys
    import numpy as np
    from scipy.spatial import Delaunay
    lib = C.CDLL(sys.argv[1])
    P = C.c_void_p
    lib.gs_delaunay.argtypes = [P, C.c_int32, P, C.c_int32, P]
    lib.gs_delaunay.restype = C.c_int

    def tri(pts):
        pts = np.ascontiguousarray(pts, dtype=np.int32)
        n = pts.shape[0]
        cap = max(2 * n, 8)
        out = np.zeros((cap, 3), np.int32)
        cnt = np.zeros(1, np.int32)
        st = lib.gs_delaunay(pts.ctypes.data, n, out.ctypes.data, cap, cnt.ctypes.data)
        return st, out[:cnt[0]]

    def orient(p, t):
        a, b, c = p[t[:, 0]].astype(np.int64), p[t[:, 1]].astype(np.int64), p[t[:, 2]].astype(np.int64)
        return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])

    rng = np.random.default_rng(5)
    for n in (3, 4, 17, 200, 3000):
        pts = rng.choice(4096 * 4096, n, replace=False)
        pts = np.stack([pts % 4096, pts // 4096], 1)
        st, t = tri(pts)
        assert st == 0, st
        assert np.all(orient(pts, t) > 0)
        ref = Delaunay(pts.astype(np.float64)).simplices
        assert t.shape[0] == ref.shape[0], (n, t.shape, ref.shape)
        key = lambda s: sorted(tuple(sorted(x)) for x in s.tolist())
        assert key(t) == key(ref), n
    g = np.stack(np.meshgrid(np.arange(0, 60, 3), np.arange(0, 45, 3)), -1).reshape(-1, 2)
    st, t = tri(g)
    assert st == 0 and np.all(orient(g, t) > 0)
    area = orient(g, t).sum()
    assert area == 2 * 57 * 42, area  # the triangles tile the hull exactly
    for bad in ([[1, 1], [2, 5], [1, 1], [7, 3]], [[0, 0], [1, 1], [2, 2], [5, 5]], [[0, 0], [40000, 1], [2, 9]]):
        st, _ = tri(np.array(bad))
        assert st != 0
    print("delaunay ok")
""")


def test_delaunay_under_sanitizers(tmp_path):
    pytest.importorskip("scipy")
    stub = tmp_path / "fail_stub.cpp"
    stub.write_text(_DELAUNAY_STUB)
    lib = str(tmp_path / "libdelaunay_san.so")
    _build(lib, [os.path.join(ROOT, "paper_2409_13055_amd", "csrc", "delaunay.cpp"), str(stub)],
           ["-I" + os.path.join(ROOT, "include")])
    drv = tmp_path / "drive.py"
    drv.write_text(_DELAUNAY_DRIVER)
    r = subprocess.run([sys.executable, str(drv), lib], cwd=ROOT, env=_env(), capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "delaunay ok" in r.stdout
