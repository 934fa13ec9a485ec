"""Host logic of the library (tree planner lists and colour classes, device
pool size classes), checked on the CPU by tests/host/host_checks.cpp against
brute-force definitions. The program is built by __graft_entry__.build(); it
is built here only if it is missing."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "host", "host_checks")


def test_planner_and_pool_host_checks():
    if not os.path.exists(EXE):
        from paper_1508_01835_amd import build as b
        b.build_host_checks()
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
