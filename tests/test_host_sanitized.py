"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer,
with the library's BP_DEBUG checks (tests/host/host_runtime.cpp, built by
paper_1010_0012_amd/build.py build_sanitized): argument checks of every
entry point, potential tables, workspace / gradient / multi-scale /
sparse-table layouts, batch descriptors and the factor-graph build.  Runs on
machines without a GPU only (the program hands the library host addresses
in place of device buffers)."""
import os
import subprocess

import pytest


def _gpu_present():
    if os.path.exists("/dev/kfd"):
        return True
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="the sanitized host check runs where there is no GPU")
def test_host_runtime_under_sanitizers():
    from paper_1010_0012_amd import build
    prog = build.build_sanitized()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([prog], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out and "BP_ASSERT" not in out, out[-4000:]
    assert " 0 failures" in out, out[-2000:]
