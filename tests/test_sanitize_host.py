"""The library's host code (tile planner and its qubit search, block fusion,
partial-amplitude cuts, the script reader, the single-amplitude graph and
elimination order) under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize/build.sh builds tests/sanitize/host_driver.cpp against the
sources with both sanitizers on the host side, and the driver's planning
runs (valid and malformed inputs) must finish without a finding.  No device
is used."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_planners_clean_under_asan_and_ubsan(tmp_path):
    out = tmp_path / "asan"
    subprocess.run(["bash", os.path.join(HERE, "sanitize", "build.sh"), str(out)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(out / "host_driver")], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
