"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its pins
and the gradient oracle's tests run in a child process that loads the
sanitizer build of liboracle, and every finding is fatal."""
import os
import subprocess
import sys

import oracle.binding as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_clean_under_sanitizers():
    ob.build_oracle(sanitize=True)
    env = ob.sanitizer_env()
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "tests/test_oracle_pins.py", "tests/test_nms_oracle.py", "-k", "not planted"]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert " passed" in out and "failed" not in out, out[-2000:]
