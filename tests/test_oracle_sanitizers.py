"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a C driver runs R-MAT generation, exact and FN-Approx walks
with counts and checksum, the cost model and the gap decision at extreme
sizes; any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "drv"
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
             "-fsanitize=address,undefined"]
    subprocess.check_call(["gcc"] + flags + [os.path.join(ROOT, "oracle", "oracle.c"),
                                             os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
                                             "-o", str(exe), "-lpthread", "-lm"])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.splitlines()
    assert len(lines) == 14
    # p = q = 1: FN-Approx draws what the exact rule draws (same checksum)
    sums = {}
    for ln in lines:
        if ln.startswith("weighted="):
            f = dict(kv.split("=") for kv in ln.split())
            sums[(f["weighted"], f["p"], f["q"], f["T"])] = f["checksum"]
    for wtd in ("0", "1"):
        assert sums[(wtd, "1", "1", "0")] == sums[(wtd, "1", "1", "100")]
    assert sums[("0", "2", "0.5", "0")] != sums[("0", "2", "0.5", "100")]
