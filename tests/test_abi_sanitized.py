"""The host side of the C-ABI library (description validation, planning, the
identical-block and symmetry checks, handle checks) built with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code, driven in a child process with the
sanitizer runtime preloaded through every check of test_abi_cpu: the corrupted and
malformed descriptions, bad scalars and options, unknown handles, and the plans of
generated descriptions (stored-once near blocks, symmetric near blocks and couplings,
mixed leaf depths).  Every call must return its documented status and no sanitizer
may report."""
import glob
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
ROOT = sys.argv[1]
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
from paper_1703_01175_amd import _lib
_lib.LIB_PATH = sys.argv[2]
import test_abi_cpu as T
from conftest import built
lib = _lib.load()
assert lib._name == sys.argv[2], lib._name
T.test_exports_every_declared_symbol()
desc = built("rod")[1]
T.test_plan_ok(desc)
T.test_plan_reserves_partials_only_for_symmetric_near_blocks(desc)
T.test_plan_stores_identical_near_blocks_once()
T.test_plan_keeps_near_blocks_when_few_repeat()
T.test_plan_reserves_coupling_partials_only_for_symmetric_couplings()
for field, fn, status in T.CORRUPTIONS:
    T.test_corrupted_descriptions_rejected(desc, field, fn, status)
T.test_bad_scalars_and_options(desc)
T.test_bad_handles_without_gpu()
for name in ("cube12", "cube13", "box9", "slab_sym"):
    st, n = T._plan(built(name)[1], max_rhs=4, tiers=7)
    assert st == 0 and n > 0, (name, st)
print("sanitized host checks passed", flush=True)
"""


def _runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


def test_host_code_under_address_and_ub_sanitizers():
    rt = _runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    from paper_1703_01175_amd.build import ASAN_LIB, build
    build(sanitize=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, ASAN_LIB], capture_output=True, text=True, env=env,
                       timeout=900)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized host checks passed" in r.stdout, report
