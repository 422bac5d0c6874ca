"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/build_host_check.py builds every library source with both sanitizers on the host half
(device code unchanged) and links tests/native/host_check.cpp against the objects.  On the CPU the
driver runs the entry points that never touch the GPU (colouring, argument checks, workspace
sizing); on the GPU it drives every entry point (all valid solver configurations, batched solves,
the serving loop, kernel-level calls, documented error returns) and recomputes each reported
residual on the host.  A sanitizer finding or a failed check gives a non-zero exit status."""
import importlib.util
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("build_host_check", os.path.join(HERE, "native", "build_host_check.py"))
HC = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(HC)


def _run(exe, phase, timeout):
    r = subprocess.run([exe, phase], capture_output=True, text=True, timeout=timeout, env=HC.run_env())
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "host check passed" in r.stdout and "FAIL" not in r.stdout, out[-4000:]
    return out


def test_host_check_cpu_phase(tmp_path):
    exe = HC.build(str(tmp_path))
    out = _run(exe, "cpu", 300)
    assert "cpu phase:" in out


@pytest.mark.gpu
def test_host_check_gpu_phase():
    """Runs the executable that build() left in tests/native/_build (nothing is compiled here);
    it must have been built from the current sources."""
    why = HC.stale_reason()
    assert why is None, why + " (run __graft_entry__.build() or tests/native/build_host_check.py)"
    out = _run(os.path.join(HC.DEFAULT_OUT, "host_check"), "gpu", 110)
    assert "solver configurations:" in out and "not converged 0" in out
