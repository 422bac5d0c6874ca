"""C-ABI contract checks that need no GPU: the library loads, exports every
function the public headers declare, sizes its workspace, and rejects bad
configurations before touching the device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_1807_09467_amd import rsolve, serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(rsolve_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rsolve.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return rsolve.load()


def test_headers_declare_the_binding_exports():
    assert set(declared_functions()) == set(rsolve.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_struct_layouts():
    assert ctypes.sizeof(rsolve.Config) == 56
    assert ctypes.sizeof(rsolve.CSR) == 48
    assert ctypes.sizeof(rsolve.Stats) == 64


C_LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "rsolve_server.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(rsolve_config), sizeof(rsolve_csr),
           sizeof(rsolve_stats), sizeof(rsolve_batch_solve_item), offsetof(rsolve_batch_solve_item, status),
           offsetof(rsolve_batch_solve_item, stats), sizeof(rsolve_batch_update_item),
           sizeof(rsolve_prof_entry), sizeof(rsolve_server_config), sizeof(rsolve_completion),
           sizeof(rsolve_server_info), sizeof(rsolve_spmv_shape));
    return 0;
}
"""


def test_struct_layouts_match_the_c_compiler(tmp_path):
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "probe.c"
    src.write_text(C_LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(rsolve.Config), ctypes.sizeof(rsolve.CSR), ctypes.sizeof(rsolve.Stats),
            ctypes.sizeof(rsolve.BatchSolveItem), rsolve.BatchSolveItem.status.offset,
            rsolve.BatchSolveItem.stats.offset, ctypes.sizeof(rsolve.BatchUpdateItem),
            ctypes.sizeof(rsolve.ProfEntry), ctypes.sizeof(serve.ServerConfig), ctypes.sizeof(serve.Completion),
            ctypes.sizeof(serve.ServerInfo), ctypes.sizeof(rsolve.SpmvShape)]
    assert got == want


def test_server_calls_reject_bad_arguments(lib):
    serve._lib()
    h = ctypes.c_void_p()
    assert lib.rsolve_server_create(None, ctypes.byref(h)) == rsolve.E_INVALID
    cfg = serve.ServerConfig(None, 1 << 20, 2, 64, 16, 1)          # no pool
    assert lib.rsolve_server_create(ctypes.byref(cfg), ctypes.byref(h)) == rsolve.E_INVALID
    cfg = serve.ServerConfig(0x1001, 1 << 20, 2, 64, 16, 1)        # misaligned pool
    assert lib.rsolve_server_create(ctypes.byref(cfg), ctypes.byref(h)) == rsolve.E_INVALID
    cfg = serve.ServerConfig(0x100000, 1 << 20, 0, 64, 16, 1)      # no large worker
    assert lib.rsolve_server_create(ctypes.byref(cfg), ctypes.byref(h)) == rsolve.E_INVALID
    cfg = serve.ServerConfig(0x100000, 1 << 20, 2, 257, 16, 1)     # batch above the launch limit
    assert lib.rsolve_server_create(ctypes.byref(cfg), ctypes.byref(h)) == rsolve.E_INVALID
    assert not h.value
    cnt = ctypes.c_int32()
    assert lib.rsolve_server_poll(None, None, 0, ctypes.byref(cnt), 0) == rsolve.E_INVALID
    assert lib.rsolve_server_close(None, 1) == rsolve.E_INVALID
    assert lib.rsolve_server_destroy(None) == rsolve.E_INVALID


def test_serving_specs_are_seeded_and_in_range():
    a = serve.serving_specs(64, seed=3)
    b = serve.serving_specs(64, seed=3)
    assert a == b and serve.serving_specs(64, seed=4) != a
    arr = [s.arrival_s for s in a]
    assert all(x < y for x, y in zip(arr, arr[1:]))
    assert {s.p for s in a} <= {1, 2, 3} and all(64 <= s.N <= 384 and s.N % 32 == 0 for s in a)
    assert all(1e-4 <= s.eps <= 1e-1 and 10 <= s.steps <= 60 for s in a)
    # mean inter-arrival near 1 / rate
    gaps = np.diff([0.0] + [s.arrival_s for s in serve.serving_specs(4000, rate=200.0, seed=1)])
    assert abs(gaps.mean() - 5e-3) < 5e-4


def test_batch_calls_reject_bad_arrays(lib):
    assert lib.rsolve_solve_batch(None, 1, None) == rsolve.E_INVALID
    assert lib.rsolve_solve_batch(None, -1, None) == rsolve.E_INVALID
    assert lib.rsolve_update_recycle_batch(None, 2, None) == rsolve.E_INVALID
    # an empty batch is a no-op that needs no device
    assert lib.rsolve_solve_batch(None, 0, None) == rsolve.OK
    assert lib.rsolve_update_recycle_batch(None, 0, None) == rsolve.OK


def test_workspace_bytes_valid_and_monotone(lib):
    cfg = rsolve.make_config(restart_m=30, recycle_k=5, snapshots_s=10)
    a = rsolve.workspace_bytes(cfg, 1089, 8409)
    b = rsolve.workspace_bytes(cfg, 4225, 37249)
    assert 0 < a < b and a % 256 == 0
    big = rsolve.make_config(restart_m=50, recycle_k=16, snapshots_s=32)
    assert rsolve.workspace_bytes(big, 1089, 8409) > a
    # mixed precision keeps float32 copies of the Krylov basis instead of float64
    fp64 = rsolve.workspace_bytes(rsolve.make_config(restart_m=50, recycle_k=16, snapshots_s=32, precond="jacobi"),
                                  2362369, 58789033)
    ir = rsolve.workspace_bytes(rsolve.make_config(restart_m=50, recycle_k=16, snapshots_s=32, precond="jacobi",
                                                   precision="fp32_ir"), 2362369, 58789033)
    assert ir < fp64 < 4 * 2 ** 30


@pytest.mark.parametrize("bad", [
    dict(restart_m=0), dict(restart_m=129), dict(recycle_k=65, snapshots_s=65), dict(recycle_k=5, snapshots_s=3),
    dict(svd_interval=0), dict(max_iters=0), dict(precision="fp32_ir", inner_tol=0.0),
    dict(precision="fp32_ir", inner_tol=1.0),
])
def test_invalid_configs_rejected(lib, bad):
    kw = dict(restart_m=30)
    kw.update(bad)
    cfg = rsolve.make_config(**kw)
    assert rsolve.workspace_bytes(cfg, 100, 500) == 0
    h = ctypes.c_void_p()
    rc = lib.rsolve_create_sequence(ctypes.byref(cfg), 100, 500, None, None, 0, ctypes.byref(h))
    assert rc == rsolve.E_INVALID and not h.value


def test_method_and_select_values(lib):
    """Methods 0..5, 9 and 10 (plain, the oblique, orthogonal and least-squares rows of Table 1,
    projection guess) and both mode selections are accepted; values outside are refused."""
    for m in ("plain", "aug_oblique", "defl_oblique", "aug_ortho", "defl_ortho", "guess_project", "aug_ls",
              "defl_ls"):
        for sel in ("largest", "smallest"):
            assert rsolve.workspace_bytes(rsolve.make_config(restart_m=30, recycle_k=4, snapshots_s=6, method=m,
                                                             select=sel), 100, 500) > 0
    for field, v in (("method", 11), ("method", -1), ("select", 2)):
        cfg = rsolve.make_config(restart_m=30)
        setattr(cfg, field, v)
        assert rsolve.workspace_bytes(cfg, 100, 500) == 0


@pytest.mark.parametrize("order", [2, 3, 4])
def test_extrapolation_configs(lib, order):
    """Extrapolation of order q (eqs. (ext2)-(ext4)) needs a ring of at least q solutions and no
    recycle space; its workspace holds the ring (s vectors) and grows with s."""
    m = "guess_extrap%d" % order
    ok = rsolve.workspace_bytes(rsolve.make_config(restart_m=30, snapshots_s=order, method=m), 1000, 5000)
    big = rsolve.workspace_bytes(rsolve.make_config(restart_m=30, snapshots_s=order + 4, method=m), 1000, 5000)
    plain = rsolve.workspace_bytes(rsolve.make_config(restart_m=30, method="plain"), 1000, 5000)
    assert ok > plain and big - ok >= 4 * 1000 * 8
    assert rsolve.workspace_bytes(rsolve.make_config(restart_m=30, snapshots_s=order - 1, method=m), 1000, 5000) == 0
    assert rsolve.workspace_bytes(rsolve.make_config(restart_m=30, recycle_k=2, snapshots_s=order + 2, method=m),
                                  1000, 5000) == 0


def test_ortho_field(lib):
    """The orthogonalisation scheme is 0 (CGS2) or 1 (delayed); anything else is refused."""
    ok = rsolve.make_config(restart_m=30, ortho="dcgs2")
    assert ok.ortho == 1 and rsolve.workspace_bytes(ok, 100, 500) > 0
    for v in (2, -1):
        cfg = rsolve.make_config(restart_m=30)
        cfg.ortho = v
        assert rsolve.workspace_bytes(cfg, 100, 500) == 0


def test_bad_sizes_and_workspace(lib):
    cfg = rsolve.make_config()
    assert rsolve.workspace_bytes(cfg, 0, 10) == 0
    assert rsolve.workspace_bytes(cfg, 100, 50) == 0     # nnz < n
    h = ctypes.c_void_p()
    rc = lib.rsolve_create_sequence(ctypes.byref(cfg), 100, 500, None, None, 0, ctypes.byref(h))
    assert rc == rsolve.E_WORKSPACE
    assert b"workspace" in lib.rsolve_last_error()
    # a misaligned workspace pointer is refused before any device call
    rc = lib.rsolve_create_sequence(ctypes.byref(cfg), 100, 500, None, ctypes.c_void_p(0x1001), 1 << 30,
                                    ctypes.byref(h))
    assert rc == rsolve.E_WORKSPACE


def test_null_handles_rejected(lib):
    st = rsolve.Stats()
    assert lib.rsolve_solve(None, None, None, None, None, 1e-8, ctypes.byref(st)) == rsolve.E_INVALID
    assert lib.rsolve_update_recycle(None, None) == rsolve.E_INVALID
    assert lib.rsolve_destroy_sequence(None) == rsolve.E_INVALID
    assert lib.rsolve_get_recycle(None, None, None, None, 0, None, 0) == rsolve.E_INVALID
    assert lib.rsolve_kernel_workspace_bytes(0, 4) == 0
    assert lib.rsolve_kernel_workspace_bytes(100, 65) == 0


def test_status_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.rsolve_status_string(code)
    assert lib.rsolve_status_string(12345) == b"unknown status"


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the library missing, load() raises instead of computing anything elsewhere."""
    monkeypatch.setattr(rsolve, "_lib", None)
    monkeypatch.setattr(rsolve, "LIB_PATH", str(tmp_path / "librsolve.so"))
    with pytest.raises(RuntimeError, match="not built"):
        rsolve.load()


def test_binding_refuses_host_tensors():
    """Arguments must be device tensors of the right type, size and layout; nothing is copied silently."""
    import torch
    with pytest.raises(TypeError, match="CUDA"):
        rsolve._ptr(torch.zeros(4, dtype=torch.float64), torch.float64, 4, "b")
    with pytest.raises(TypeError, match="CUDA"):
        rsolve._ptr(torch.zeros(4, dtype=torch.float32), torch.float64, 4, "b")
