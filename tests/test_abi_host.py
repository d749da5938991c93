"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid parameters before touching a device."""
import math
import os
import re

import pytest

import paper_1809_10186_amd as qc
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qcoll.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qcoll_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = qc.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    L = qc.lib()
    for code, name in qc.STATUS.items():
        assert L.qcoll_status_str(code).decode() == name
    assert L.qcoll_version() >= 1


def ok_kw(**over):
    kw = dict(N=16, L=6.0, N_rho=8, sphere=W.sphere_rule(12), omega=0.81, prefactor=None,
              svd_rank=-1, svd_tol=0.0, precision=qc.QCOLL_FP32)
    kw.update(over)
    return kw


def test_valid_params_pass():
    code, _ = qc.params_check(**ok_kw())
    assert code == 0
    assert qc.params_check(**ok_kw(sphere=None))[0] == 0
    assert qc.params_check(**ok_kw(svd_rank=0, svd_tol=1e-8))[0] == 0
    for N in (8, 12, 24, 32, 48, 64):
        assert qc.params_check(**ok_kw(N=N))[0] == 0
    for a in (1.2, 1.5, 2.0):    # VSS kernels with the full table
        assert qc.params_check(**ok_kw(alpha=a))[0] == 0
    assert qc.params_check(**ok_kw(nyquist="literal"))[0] == 0
    assert qc.params_check(**ok_kw(nyquist="literal", svd_rank=0, svd_tol=1e-6))[0] == 0


@pytest.mark.parametrize("over,code,frag", [
    (dict(N=0), 1, "N"), (dict(N=15), 1, "even"), (dict(N=20), 2, "one of"), (dict(N=96), 2, "one of"),
    (dict(N=64, alpha=1.5), 2, "VSS"),
    (dict(L=0.0), 1, "L"), (dict(L=float("nan")), 1, "L"), (dict(L=-1.0), 1, "L"),
    (dict(N_rho=0), 1, "N_rho"), (dict(N_rho=65), 2, "N_rho"),
    (dict(omega=0.4), 1, "omega"), (dict(omega=1.2), 1, "omega"),
    (dict(alpha=1.5, svd_rank=0, svd_tol=1e-8), 2, "VSS"), (dict(alpha=3.0), 1, "alpha"),
    (dict(alpha=0.9), 1, "alpha"),
    (dict(precision=7), 1, "precision"),
    (dict(svd_rank=0, svd_tol=0.0), 1, "svd_tol"), (dict(svd_rank=99), 1, "svd_rank"),
    (dict(prefactor=float("inf")), 1, "prefactor"),
    (dict(nyquist=2), 1, "nyquist"), (dict(nyquist="literal", alpha=1.5), 2, "literal"),
])
def test_invalid_params_rejected(over, code, frag):
    c, msg = qc.params_check(**ok_kw(**over))
    assert c == code
    assert frag in msg


def test_invalid_sphere_rules():
    pts, w = W.sphere_rule(6)
    bad_w = w.copy()
    bad_w[0] *= 2
    assert qc.params_check(**ok_kw(sphere=(pts, bad_w)))[0] == 1
    bad_p = pts.copy()
    bad_p[1] *= 1.01
    assert qc.params_check(**ok_kw(sphere=(bad_p, w)))[0] == 1
    neg = w.copy()
    neg[0], neg[1] = -neg[0], neg[1] + 2 * neg[0]
    assert qc.params_check(**ok_kw(sphere=(pts, neg)))[0] == 1


def test_builtin_rule_is_the_icosahedral_one():
    # the built-in rule is used when no table is passed; M other than 6 is rejected then
    p, keep = qc.make_params(16, 6.0, 8, None, 0.81)
    p.M = 12
    import ctypes
    assert qc.lib().qcoll_params_check(ctypes.byref(p)) == 1
    assert math.isclose(sum(W.sphere_rule(6)[1]), 2 * math.pi)


def test_qcoll_log_reports_argument_errors():
    """QCOLL_LOG=1 turns on the library's stderr diagnostics (read once per
    process); argument errors are reported there as well as by qcoll_last_error."""
    import subprocess
    import sys
    code = ("import paper_1809_10186_amd as qc, workloads as W; "
            "print(qc.params_check(N=15, L=6.0, N_rho=8, sphere=W.sphere_rule(12), omega=0.81)[0])")
    env = dict(os.environ, QCOLL_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"
    assert "[qcoll] error: N must be a positive even integer" in r.stderr
    env["QCOLL_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert "[qcoll]" not in r.stderr
