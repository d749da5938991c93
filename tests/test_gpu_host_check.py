"""The host-sanitized self-check (tests/host_check/qcoll_host_check.cpp, built by
__graft_entry__.build() with AddressSanitizer and UndefinedBehaviorSanitizer on
the host code of the validation layer, plan precompute, autotune-cache parser
and group / 1-D driver set-up): it must run clean on the GPU."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "host_check", "qcoll_host_check")


def test_host_sanitized_self_check(tmp_path):
    assert os.path.exists(BIN), "tests/host_check/qcoll_host_check is missing: run __graft_entry__.build()"
    env = dict(os.environ)
    # the harness may preload a library of its own ahead of the sanitizer runtime
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    env.pop("QCOLL_AUTOTUNE_CACHE", None)
    r = subprocess.run([BIN, str(tmp_path / "tune_cache.txt")], env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.returncode == 0
    assert "qcoll host check: ok" in r.stdout
