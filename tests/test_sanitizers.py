"""The FP64 oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a driver (tests/sanitize_oracle_driver.c) exercises its
entry points in 2D and 3D for both pair potentials and both lattices,
including the error paths; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(HERE, "sanitize_oracle_driver.c"),
           os.path.join(ROOT, "oracle", "pic_oracle.c"), "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    # the environment is passed on as it is; ASan is told not to insist on
    # coming first among preloaded libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "oracle sanitizer driver ok" in r.stdout
