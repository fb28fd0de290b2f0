"""The oracle's pins again, against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (host code only, no GPU).

A child pytest process preloads the ASan runtime and loads the sanitized
library through SHOCK_ORACLE_LIB; any out-of-bounds access, use after free,
signed overflow, misaligned load or shift out of range in the oracle aborts
it.  The heaviest statistical pins are left out to keep the run short.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PIN_FILES = [
    "tests/test_oracle_pins.py", "tests/test_oracle_verify_pins.py", "tests/test_oracle_rf_pins.py",
    "tests/test_oracle_code_pins.py", "tests/test_oracle_mphf_pins.py", "tests/test_oracle_bip_pins.py",
    "tests/test_graph_rules.py",
]


def test_oracle_pins_under_sanitizers(tmp_path):
    import oracle
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime is not installed")
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env.update(SHOCK_ORACLE_LIB=so, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
           "-k", "not ideal_hashing and not matches_ideal and not uniform", *PIN_FILES]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, tail
