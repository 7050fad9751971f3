"""The C ABI walked by tests/abi_check.cpp, with the library's host code built under
AddressSanitizer and UndefinedBehaviorSanitizer (host only; the kernels are the ordinary
gfx950 code objects).  On the CPU: the calls that fail before any device work (option
validation, calls out of order, malformed run-state records).  On the GPU: every family
of calls on a three-body problem, including truncated and corrupted run-state records,
overlapping poses, the learned warm start and the low-level sums."""
import os
import subprocess

import pytest

from paper_1606_07428_amd import build as rbm_build


def _binary():
    if not os.path.exists(rbm_build.ABI_CHECK):
        rbm_build.build(verbose=False)
    return rbm_build.ABI_CHECK


def _run(args, timeout):
    r = subprocess.run([_binary()] + args, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    print(out, flush=True)
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert r.returncode == 0 and out.rstrip().endswith("abi_check: ok"), out[-2000:]


def test_host_paths_under_sanitizers():
    _run(["--host"], 60)


@pytest.mark.gpu
def test_abi_walk_under_host_sanitizers():
    print("\n[case] abi_check: three bodies p=6, every family of calls, host ASan + UBSan", flush=True)
    _run([], 110)
