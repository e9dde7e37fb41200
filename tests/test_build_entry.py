"""__graft_entry__.build() end to end on the CPU: every HIP source compiles for gfx950, the oracle
compiles, and the library it leaves loads with the ABI version the bindings expect."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_entry_point_builds_and_loads():
    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.build(); print('built')"], cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "built" in r.stdout
