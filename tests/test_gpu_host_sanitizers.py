"""The C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/host_sanitize_driver is liboct's sources and a C++ driver
linked into one executable whose HOST code is instrumented (the device code is
built as usual; build() makes it).  The driver calls every entry point, valid
and invalid, on B-scans (50% mask and batch 2, ragged sizes, the literal
model) and a volume: plan creation and destruction and release, the
operators, prox for every penalty, the power iteration, solves for every
penalty with the objective report, a resumed solve, per-item weights, every
stage, every direct image, both NCC calls, and argument errors.  It exits 0
only if every status is the documented one; any sanitizer report (heap or
stack misuse, undefined behaviour, leaks from our own allocations) aborts it.
"""
import os
import subprocess

import pytest

from gpu_util import flush

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "sanitize", "host_sanitize_driver")
SUPP = os.path.join(HERE, "sanitize", "lsan_runtime.supp")


def test_c_abi_under_host_sanitizers():
    assert os.path.exists(EXE), f"{EXE} is missing: run __graft_entry__.build()"
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1"
    env["LSAN_OPTIONS"] = f"suppressions={SUPP}:print_suppressions=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    flush("[sanitize] running the instrumented driver")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=600, env=env)
    print(r.stderr[-6000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("PASS"), r.stdout
