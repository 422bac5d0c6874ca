"""ctypes binding of librsolve.so, the C-ABI declared in include/rsolve.h and
include/rsolve_kernels.h.

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace and the caller's
tensors) and the stream.  Importing this module does not load the library;
`load()` does, and raises if it has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsolve.so")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NONFINITE, E_WORKSPACE, E_DEVICE, E_STATE, E_BUDGET = -1, -2, -3, -4, -5, -6

PLAIN, AUG_OBLIQUE, DEFL_OBLIQUE, AUG_ORTHO, DEFL_ORTHO = 0, 1, 2, 3, 4
GUESS_PROJECT, GUESS_EXTRAP2, GUESS_EXTRAP3, GUESS_EXTRAP4 = 5, 6, 7, 8
AUG_LS, DEFL_LS = 9, 10
SELECT_LARGEST, SELECT_SMALLEST, SELECT_RITZ, SELECT_HARMONIC = 0, 1, 2, 3
PRECOND_NONE, PRECOND_JACOBI, PRECOND_SSOR = 0, 1, 2
FP64, FP32_IR = 0, 1
SAME_PATTERN = 1

FLAG_RECYCLE_DROPPED = 1
FLAG_BREAKDOWN_LUCKY = 2
FLAG_NONFINITE = 4

_METHODS = {"plain": PLAIN, "aug_oblique": AUG_OBLIQUE, "defl_oblique": DEFL_OBLIQUE, "aug_ortho": AUG_ORTHO,
            "defl_ortho": DEFL_ORTHO, "guess_project": GUESS_PROJECT, "guess_extrap2": GUESS_EXTRAP2,
            "guess_extrap3": GUESS_EXTRAP3, "guess_extrap4": GUESS_EXTRAP4, "aug_ls": AUG_LS, "defl_ls": DEFL_LS}
_SELECTS = {"largest": SELECT_LARGEST, "smallest": SELECT_SMALLEST, "ritz": SELECT_RITZ,
            "harmonic_ritz": SELECT_HARMONIC}
_PRECONDS = {"none": PRECOND_NONE, "jacobi": PRECOND_JACOBI, "ssor": PRECOND_SSOR}
_PRECISIONS = {"fp64": FP64, "fp32_ir": FP32_IR}

# every symbol the two public headers declare
EXPORTS = [
    "rsolve_workspace_bytes", "rsolve_create_sequence", "rsolve_solve", "rsolve_update_recycle",
    "rsolve_get_recycle", "rsolve_destroy_sequence", "rsolve_status_string", "rsolve_last_error",
    "rsolve_spmv", "rsolve_kernel_workspace_bytes", "rsolve_gram_tn", "rsolve_snapshot_svd",
    "rsolve_profile_enable", "rsolve_profile_read", "rsolve_solve_batch", "rsolve_update_recycle_batch",
    "rsolve_tune_spmv", "rsolve_set_spmv_shape", "rsolve_get_spmv_shape", "rsolve_enable_graphs",
    "rsolve_graph_counts", "rsolve_gram_tn_noalloc", "rsolve_colour_first_fit", "rsolve_triad",
    "rsolve_state_bytes", "rsolve_export_state", "rsolve_import_state",
    # serving loop (rsolve_server.h; bound in serve.py)
    "rsolve_server_create", "rsolve_server_open", "rsolve_server_submit", "rsolve_server_poll",
    "rsolve_server_close", "rsolve_server_info_get", "rsolve_server_destroy",
]

SMALL_MAX_RESTART, SMALL_MAX_RECYCLE, SMALL_MAX_SNAPSHOTS, SMALL_MAX_N = 64, 32, 32, 65536

PROF_KERNELS = {0: "spmv_arnoldi", 1: "dots", 2: "update_dots", 3: "update_norm"}


class Config(ctypes.Structure):
    _fields_ = [
        ("restart_m", c_int32), ("recycle_k", c_int32), ("snapshots_s", c_int32), ("svd_interval", c_int32),
        ("method", c_int32), ("precond", c_int32), ("precision", c_int32), ("max_iters", c_int32),
        ("select", c_int32), ("ortho", c_int32), ("inner_tol", c_double), ("ssor_omega", c_double),
    ]


class CSR(ctypes.Structure):
    _fields_ = [
        ("n", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p), ("col_idx", c_void_p), ("val", c_void_p),
        ("flags", c_uint32), ("reserved", c_uint32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", c_int32), ("cycles", c_int32), ("k_eff", c_int32), ("converged", c_int32),
        ("flags", c_uint32), ("its_estimate_met", c_int32), ("rel_res_true", c_double),
        ("rel_res_implicit", c_double),
        ("t_setup_ms", c_double), ("t_cycles_ms", c_double), ("t_total_ms", c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ProfEntry(ctypes.Structure):
    _fields_ = [("kernel", c_int32), ("variant", c_int32), ("launches", c_int64), ("ms", c_double),
                ("bytes", c_double)]


SPMV_FORMATS = {0: "csr", 1: "banded"}


class SpmvShape(ctypes.Structure):
    _fields_ = [("lanes_per_row", c_int32), ("vec", c_int32), ("xcd_remap", c_int32), ("user_set", c_int32),
                ("format", c_int32), ("reserved", c_int32), ("us", c_double)]

    def as_dict(self):
        return {"format": SPMV_FORMATS.get(self.format, self.format), "lanes_per_row": self.lanes_per_row,
                "vec": self.vec, "xcd_remap": self.xcd_remap, "us": self.us}


class BatchSolveItem(ctypes.Structure):
    _fields_ = [("seq", c_void_p), ("A", CSR), ("b", c_void_p), ("x0", c_void_p), ("x", c_void_p), ("tol", c_double),
                ("status", c_int32), ("reserved", c_int32), ("stats", Stats)]


class BatchUpdateItem(ctypes.Structure):
    _fields_ = [("seq", c_void_p), ("x", c_void_p), ("status", c_int32), ("reserved", c_int32)]


class RsolveError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rsolve status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load librsolve.so (built in-tree by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.rsolve_workspace_bytes.argtypes = [POINTER(Config), c_int64, c_int64]
    lib.rsolve_workspace_bytes.restype = c_size_t
    lib.rsolve_create_sequence.argtypes = [POINTER(Config), c_int64, c_int64, c_void_p, c_void_p, c_size_t,
                                           POINTER(c_void_p)]
    lib.rsolve_create_sequence.restype = c_int
    lib.rsolve_solve.argtypes = [c_void_p, POINTER(CSR), c_void_p, c_void_p, c_void_p, c_double, POINTER(Stats)]
    lib.rsolve_solve.restype = c_int
    lib.rsolve_update_recycle.argtypes = [c_void_p, c_void_p]
    lib.rsolve_update_recycle.restype = c_int
    lib.rsolve_get_recycle.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_double), c_int32,
                                       c_void_p, c_int64]
    lib.rsolve_get_recycle.restype = c_int
    lib.rsolve_state_bytes.argtypes = [c_void_p]
    lib.rsolve_state_bytes.restype = c_size_t
    lib.rsolve_export_state.argtypes = [c_void_p, c_void_p, c_size_t, POINTER(c_size_t)]
    lib.rsolve_export_state.restype = c_int
    lib.rsolve_import_state.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.rsolve_import_state.restype = c_int
    lib.rsolve_destroy_sequence.argtypes = [c_void_p]
    lib.rsolve_destroy_sequence.restype = c_int
    lib.rsolve_status_string.argtypes = [c_int]
    lib.rsolve_status_string.restype = c_char_p
    lib.rsolve_last_error.argtypes = []
    lib.rsolve_last_error.restype = c_char_p
    lib.rsolve_spmv.argtypes = [POINTER(CSR), c_void_p, c_void_p, c_void_p]
    lib.rsolve_spmv.restype = c_int
    lib.rsolve_kernel_workspace_bytes.argtypes = [c_int64, c_int32]
    lib.rsolve_kernel_workspace_bytes.restype = c_size_t
    lib.rsolve_gram_tn.argtypes = [c_int64, c_void_p, c_int64, c_int32, c_void_p, c_int64, c_int32,
                                   POINTER(c_double), c_void_p, c_size_t, c_void_p]
    lib.rsolve_gram_tn.restype = c_int
    lib.rsolve_gram_tn_noalloc.argtypes = [c_int64, c_void_p, c_int64, c_int32, c_void_p, c_int64, c_int32,
                                           POINTER(c_double), c_void_p]
    lib.rsolve_gram_tn_noalloc.restype = c_int
    lib.rsolve_colour_first_fit.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, POINTER(c_int32)]
    lib.rsolve_colour_first_fit.restype = c_int
    lib.rsolve_triad.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_double, c_void_p]
    lib.rsolve_triad.restype = c_int
    lib.rsolve_snapshot_svd.argtypes = [c_int64, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int64,
                                        POINTER(c_double), POINTER(c_int32), POINTER(c_int32), c_void_p, c_size_t,
                                        c_void_p]
    lib.rsolve_snapshot_svd.restype = c_int
    lib.rsolve_profile_enable.argtypes = [c_void_p, c_int32]
    lib.rsolve_profile_enable.restype = c_int
    lib.rsolve_profile_read.argtypes = [c_void_p, POINTER(ProfEntry), c_int32, POINTER(c_int32), c_int32]
    lib.rsolve_profile_read.restype = c_int
    lib.rsolve_tune_spmv.argtypes = [c_void_p, POINTER(CSR), c_int32, POINTER(SpmvShape), c_int32, POINTER(c_int32)]
    lib.rsolve_tune_spmv.restype = c_int
    lib.rsolve_set_spmv_shape.argtypes = [c_void_p, POINTER(SpmvShape)]
    lib.rsolve_set_spmv_shape.restype = c_int
    lib.rsolve_get_spmv_shape.argtypes = [c_void_p, POINTER(SpmvShape)]
    lib.rsolve_get_spmv_shape.restype = c_int
    lib.rsolve_enable_graphs.argtypes = [c_void_p, c_int32]
    lib.rsolve_enable_graphs.restype = c_int
    lib.rsolve_graph_counts.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
    lib.rsolve_graph_counts.restype = c_int
    lib.rsolve_solve_batch.argtypes = [POINTER(BatchSolveItem), c_int32, c_void_p]
    lib.rsolve_solve_batch.restype = c_int
    lib.rsolve_update_recycle_batch.argtypes = [POINTER(BatchUpdateItem), c_int32, c_void_p]
    lib.rsolve_update_recycle_batch.restype = c_int
    _lib = lib
    return lib


def _check(status, allow=(OK,)):
    if status in allow:
        return status
    lib = load()
    raise RsolveError(status, f"{lib.rsolve_status_string(status).decode()}: {lib.rsolve_last_error().decode()}")


_ORTHOS = {"cgs2": 0, "dcgs2": 1}


def make_config(restart_m=30, recycle_k=0, snapshots_s=0, svd_interval=1, method="aug_oblique", precond="none",
                precision="fp64", max_iters=10000, inner_tol=1e-5, ortho="cgs2", select="largest",
                ssor_omega=1.0) -> Config:
    return Config(restart_m, recycle_k, snapshots_s, svd_interval, _METHODS[method], _PRECONDS[precond],
                  _PRECISIONS[precision], max_iters, _SELECTS[select], _ORTHOS[ortho], float(inner_tol),
                  float(ssor_omega))


def workspace_bytes(cfg: Config, n: int, nnz_max: int) -> int:
    return int(load().rsolve_workspace_bytes(byref(cfg), n, nnz_max))


def _ptr(t, dtype, numel=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} entries, got {t.numel()}")
    return t.data_ptr()


def _stream_handle(stream):
    return c_void_p(stream.cuda_stream) if stream is not None else c_void_p(0)


class Sequence:
    """One time-stepping sequence (rsolve_create_sequence ... rsolve_destroy_sequence)."""

    def __init__(self, n, nnz_max, device=None, stream=None, **cfg):
        import torch
        self.lib = load()
        self.cfg = make_config(**cfg)
        self.n = int(n)
        self.nnz_max = int(nnz_max)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = workspace_bytes(self.cfg, self.n, self.nnz_max)
        if nbytes == 0:
            raise RsolveError(E_INVALID, "invalid configuration or sizes")
        self.workspace_bytes = nbytes
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.rsolve_create_sequence(byref(self.cfg), self.n, self.nnz_max,
                                                   _stream_handle(self.stream), c_void_p(self.ws.data_ptr()),
                                                   nbytes, byref(h)))
        self.handle = h

    def csr(self, row_ptr, col_idx, val, same_pattern=False):
        import torch
        n = self.n
        nnz = int(val.numel())
        return CSR(n, nnz, _ptr(row_ptr, torch.int32, n + 1, "row_ptr"), _ptr(col_idx, torch.int32, nnz, "col_idx"),
                   _ptr(val, torch.float64, nnz, "val"), SAME_PATTERN if same_pattern else 0, 0)

    def solve(self, row_ptr, col_idx, val, b, x0=None, x=None, tol=1e-8, same_pattern=False, check=True):
        """Solve A x = b; returns (x, stats dict, status)."""
        import torch
        n = self.n
        A = self.csr(row_ptr, col_idx, val, same_pattern)
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=self.device)
        st = Stats()
        with torch.cuda.device(self.device):
            status = self.lib.rsolve_solve(self.handle, byref(A), c_void_p(_ptr(b, torch.float64, n, "b")),
                                           c_void_p(_ptr(x0, torch.float64, n, "x0")),
                                           c_void_p(_ptr(x, torch.float64, n, "x")), float(tol), byref(st))
        if check:
            _check(status, allow=(OK, NOT_CONVERGED))
        return x, st.as_dict(), status

    def update(self, x=None, check=True):
        import torch
        with torch.cuda.device(self.device):
            status = self.lib.rsolve_update_recycle(self.handle, c_void_p(_ptr(x, torch.float64, self.n, "x")))
        if check:
            _check(status)
        return status

    def recycle(self, with_basis=False):
        import torch
        k = c_int32()
        r = c_int32()
        cap = 64
        sig = (c_double * cap)()
        _check(self.lib.rsolve_get_recycle(self.handle, byref(k), byref(r), sig, cap, None, 0))
        out = {"k_eff": k.value, "rank": r.value, "sigma": [sig[i] for i in range(cap)]}
        if with_basis:
            W = torch.zeros((max(k.value, 0), self.n), dtype=torch.float64, device=self.device)
            if k.value > 0:
                with torch.cuda.device(self.device):
                    _check(self.lib.rsolve_get_recycle(self.handle, byref(k), byref(r), None, 0,
                                                       c_void_p(W.data_ptr()), self.n))
            out["W"] = W
        return out

    def export_state(self):
        """The sequence's recycling state as bytes (rsolve_export_state)."""
        size = self.lib.rsolve_state_bytes(self.handle)
        buf = ctypes.create_string_buffer(size)
        written = c_size_t()
        _check(self.lib.rsolve_export_state(self.handle, buf, size, byref(written)))
        return buf.raw[:written.value]

    def import_state(self, blob, check=True):
        """Replace the recycling state with bytes from export_state (rsolve_import_state)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        status = self.lib.rsolve_import_state(self.handle, buf, len(blob))
        if check:
            _check(status)
        return status

    def tune_spmv(self, row_ptr, col_idx, val, reps=20):
        """Time every Arnoldi SpMV shape on this matrix (rsolve_tune_spmv); fastest first."""
        import torch
        A = self.csr(row_ptr, col_idx, val)
        cap = 64
        arr = (SpmvShape * cap)()
        cnt = c_int32()
        with torch.cuda.device(self.device):
            _check(self.lib.rsolve_tune_spmv(self.handle, byref(A), int(reps), arr, cap, byref(cnt)))
        return [arr[i].as_dict() for i in range(min(cnt.value, cap))]

    def set_spmv_shape(self, lanes_per_row, vec, xcd_remap=0, format="csr"):
        """format: "csr" or "banded" (rsolve.h RSOLVE_SPMV_*)."""
        fmt = {v: k for k, v in SPMV_FORMATS.items()}.get(format, format)
        _check(self.lib.rsolve_set_spmv_shape(self.handle,
                                              byref(SpmvShape(lanes_per_row, vec, xcd_remap, 0, fmt, 0, 0.0))))

    def spmv_shape(self):
        sh = SpmvShape()
        _check(self.lib.rsolve_get_spmv_shape(self.handle, byref(sh)))
        d = sh.as_dict()
        d["user_set"] = bool(sh.user_set)
        return d

    def graphs(self, on=True):
        """Replay the Arnoldi steps as captured hipGraphs (rsolve_enable_graphs)."""
        _check(self.lib.rsolve_enable_graphs(self.handle, 1 if on else 0))

    def graph_counts(self):
        c, l = c_int64(), c_int64()
        _check(self.lib.rsolve_graph_counts(self.handle, byref(c), byref(l)))
        return c.value, l.value

    def profile(self, on=True, kinds=None, stride=1):
        """Per-kernel event timing: kinds = iterable of names from PROF_KERNELS (default: all);
        stride s times only every s-th step of a cycle (rsolve.h RSOLVE_PROF_STRIDE)."""
        if not on:
            mask = 0
        elif kinds is None:
            mask = 0xF
        else:
            names = {v: k for k, v in PROF_KERNELS.items()}
            mask = 0
            for k in kinds:
                mask |= 1 << names[k]
        if on:
            if not 1 <= stride <= 256:
                raise ValueError("stride must be in 1..256")
            mask |= (stride - 1) << 8
        _check(self.lib.rsolve_profile_enable(self.handle, mask))

    def profile_read(self, reset=False):
        """Per-kernel HIP-event timings: list of dicts (kernel, variant, launches, ms, bytes)."""
        cap = 32
        arr = (ProfEntry * cap)()
        cnt = c_int32()
        _check(self.lib.rsolve_profile_read(self.handle, arr, cap, byref(cnt), 1 if reset else 0))
        # with the delayed scheme, kind 1 is the two-vector sweep and kind 2 the combined update
        names = dict(PROF_KERNELS)
        if self.cfg.ortho == 1:
            names.update({1: "dots2", 2: "dcgs2_update"})
        return [{"kernel": names[arr[i].kernel], "variant": arr[i].variant, "launches": arr[i].launches,
                 "ms": arr[i].ms, "bytes": arr[i].bytes} for i in range(min(cnt.value, cap))]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.rsolve_destroy_sequence(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(jobs, stream=None, check=True):
    """One solve per job in a single batched call (rsolve_solve_batch).

    jobs: list of dicts with keys seq (Sequence), row_ptr, col_idx, val, b, and optionally x0, x,
    tol (1e-8), same_pattern (False).  Returns a list of (x, stats dict, status)."""
    import torch
    lib = load()
    items = (BatchSolveItem * max(len(jobs), 1))()
    outs = []
    for i, j in enumerate(jobs):
        seq = j["seq"]
        x = j.get("x")
        if x is None:
            x = torch.empty(seq.n, dtype=torch.float64, device=seq.device)
        outs.append(x)
        it = items[i]
        it.seq = seq.handle
        it.A = seq.csr(j["row_ptr"], j["col_idx"], j["val"], j.get("same_pattern", False))
        it.b = _ptr(j["b"], torch.float64, seq.n, "b")
        it.x0 = _ptr(j.get("x0"), torch.float64, seq.n, "x0")
        it.x = _ptr(x, torch.float64, seq.n, "x")
        it.tol = float(j.get("tol", 1e-8))
    dev = jobs[0]["seq"].device if jobs else None
    if dev is not None:
        with torch.cuda.device(dev):
            _check(lib.rsolve_solve_batch(items, len(jobs), _stream_handle(stream)))
    res = []
    for i in range(len(jobs)):
        st = items[i].status
        if check:
            _check(st, allow=(OK, NOT_CONVERGED))
        res.append((outs[i], items[i].stats.as_dict(), st))
    return res


def _item_dtype():
    """numpy view of rsolve_batch_solve_item (offsets taken from the ctypes layout)."""
    import numpy as np
    a, st = BatchSolveItem.A.offset, BatchSolveItem.stats.offset
    names, fmts, offs = [], [], []
    for name, fmt, off in [
        ("seq", "u8", BatchSolveItem.seq.offset), ("n", "i8", a + CSR.n.offset), ("nnz", "i8", a + CSR.nnz.offset),
        ("row_ptr", "u8", a + CSR.row_ptr.offset), ("col_idx", "u8", a + CSR.col_idx.offset),
        ("val", "u8", a + CSR.val.offset), ("flags", "u4", a + CSR.flags.offset), ("b", "u8", BatchSolveItem.b.offset),
        ("x0", "u8", BatchSolveItem.x0.offset), ("x", "u8", BatchSolveItem.x.offset),
        ("tol", "f8", BatchSolveItem.tol.offset), ("status", "i4", BatchSolveItem.status.offset),
        ("iterations", "i4", st + Stats.iterations.offset), ("cycles", "i4", st + Stats.cycles.offset),
        ("k_eff", "i4", st + Stats.k_eff.offset), ("converged", "i4", st + Stats.converged.offset),
        ("rel_res_true", "f8", st + Stats.rel_res_true.offset),
    ]:
        names.append(name), fmts.append(fmt), offs.append(off)
    return np.dtype({"names": names, "formats": fmts, "offsets": offs, "itemsize": ctypes.sizeof(BatchSolveItem)})


class BatchPlan:
    """A fixed set of sequences solved together round after round (one time step each per round).

    The item array is built once; each round only the value, right-hand-side, start and output
    pointers change, written through a vectorised numpy view, so the host cost per round stays
    small next to the launch.  Output vectors alternate between two buffers per sequence, so
    the previous round's solution can serve as this round's x0."""

    def __init__(self, seqs, row_ptrs, col_idxs, tol=1e-8, stream=None):
        import numpy as np
        import torch
        self.lib = load()
        self.seqs = list(seqs)
        m = len(self.seqs)
        self.items = (BatchSolveItem * max(m, 1))()
        self.view = np.frombuffer(self.items, dtype=_item_dtype(), count=m)
        self.upd = (BatchUpdateItem * max(m, 1))()
        for i, sq in enumerate(self.seqs):
            self.upd[i].seq = sq.handle
        self.view["seq"] = [sq.handle.value for sq in self.seqs]
        self.view["n"] = [sq.n for sq in self.seqs]
        self.view["row_ptr"] = [_ptr(r, torch.int32, sq.n + 1, "row_ptr") for r, sq in zip(row_ptrs, self.seqs)]
        self.view["col_idx"] = [c.data_ptr() for c in col_idxs]
        self.view["tol"] = tol
        self.out = [[torch.empty(sq.n, dtype=torch.float64, device=sq.device) for _ in range(2)] for sq in self.seqs]
        self.round = 0
        self.stream = stream
        self.device = self.seqs[0].device if self.seqs else None

    @staticmethod
    def pointers(tensors):
        """Device addresses of a list of tensors as a numpy array (precompute once per round's
        inputs to keep the per-round host work to two library calls)."""
        import numpy as np
        return np.fromiter((t.data_ptr() for t in tensors), dtype=np.uint64, count=len(tensors))

    def solve(self, vals, bs, x0s, same_pattern, nnz=None):
        """vals, bs: per-sequence device tensors, or numpy uint64 arrays of their addresses (then
        nnz gives the value counts, an int or an array); x0s: tensors (entries may be None) or
        "previous" for the outputs of the previous round.  Returns the outputs (list of tensors);
        per-item status and stats are in self.view."""
        import numpy as np
        import torch
        m = len(self.seqs)
        outs = [o[self.round & 1] for o in self.out]
        if not hasattr(self, "_outp"):
            self._outp = [self.pointers([o[0] for o in self.out]), self.pointers([o[1] for o in self.out])]
        if isinstance(vals, np.ndarray):
            self.view["val"] = vals
            self.view["nnz"] = nnz
        else:
            self.view["val"] = [v.data_ptr() for v in vals]
            self.view["nnz"] = [v.numel() for v in vals]
        self.view["b"] = bs if isinstance(bs, np.ndarray) else [b.data_ptr() for b in bs]
        if isinstance(x0s, str) and x0s == "previous":
            self.view["x0"] = self._outp[(self.round + 1) & 1]
        else:
            self.view["x0"] = [0 if x is None else x.data_ptr() for x in x0s]
        self.view["x"] = self._outp[self.round & 1]
        self.round += 1
        self.view["flags"] = SAME_PATTERN if same_pattern else 0
        with torch.cuda.device(self.device):
            _check(self.lib.rsolve_solve_batch(self.items, m, _stream_handle(self.stream)))
        bad = np.flatnonzero((self.view["status"] != OK) & (self.view["status"] != NOT_CONVERGED))
        if bad.size:
            i = int(bad[0])
            raise RsolveError(int(self.view["status"][i]), f"batch item {i} failed")
        return outs

    def update(self):
        import torch
        with torch.cuda.device(self.device):
            _check(self.lib.rsolve_update_recycle_batch(self.upd, len(self.seqs), _stream_handle(self.stream)))
        for i in range(len(self.seqs)):
            _check(self.upd[i].status)


def update_batch(seqs, xs=None, stream=None, check=True):
    """rsolve_update_recycle for every sequence in one batched call; returns the statuses."""
    import torch
    lib = load()
    items = (BatchUpdateItem * max(len(seqs), 1))()
    for i, seq in enumerate(seqs):
        items[i].seq = seq.handle
        x = xs[i] if xs is not None else None
        items[i].x = _ptr(x, torch.float64, seq.n, "x")
    if seqs:
        with torch.cuda.device(seqs[0].device):
            _check(lib.rsolve_update_recycle_batch(items, len(seqs), _stream_handle(stream)))
    out = [items[i].status for i in range(len(seqs))]
    if check:
        for st in out:
            _check(st)
    return out


def spmv(row_ptr, col_idx, val, x, y=None, stream=None):
    import torch
    lib = load()
    n = int(row_ptr.numel()) - 1
    nnz = int(val.numel())
    if y is None:
        y = torch.empty(n, dtype=torch.float64, device=x.device)
    A = CSR(n, nnz, _ptr(row_ptr, torch.int32, n + 1, "row_ptr"), _ptr(col_idx, torch.int32, nnz, "col_idx"),
            _ptr(val, torch.float64, nnz, "val"), 0, 0)
    _check(lib.rsolve_spmv(byref(A), c_void_p(_ptr(x, torch.float64, n, "x")), c_void_p(_ptr(y, torch.float64, n, "y")),
                           _stream_handle(stream)))
    return y


def _kernel_ws(n, cols, device):
    import torch
    nbytes = int(load().rsolve_kernel_workspace_bytes(n, cols))
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def gram_tn(A, B, stream=None):
    """C = A^T B for column-major tall A (p x n storage: A[c] is column c) and B; returns a numpy array."""
    import numpy as np
    lib = load()
    p, n = A.shape
    q, n2 = B.shape
    assert n == n2
    ws, nbytes = _kernel_ws(n, max(p, q), A.device)
    C = (c_double * (p * q))()
    _check(lib.rsolve_gram_tn(n, c_void_p(A.data_ptr()), n, p, c_void_p(B.data_ptr()), n, q, C,
                              c_void_p(ws.data_ptr()), nbytes, _stream_handle(stream)))
    return np.frombuffer(C, dtype=np.float64).reshape(q, p).T.copy()


def last_error():
    """The library's description of the last error seen by this thread ("" if none)."""
    return load().rsolve_last_error().decode()


def triad(a, b, c, s, stream=None):
    """a = b + s c on the device (float64 CUDA tensors of one length), asynchronous."""
    import torch
    n = a.numel()
    _check(load().rsolve_triad(n, c_void_p(_ptr(a, torch.float64, n, "a")), c_void_p(_ptr(b, torch.float64, n, "b")),
                               c_void_p(_ptr(c, torch.float64, n, "c")), float(s), _stream_handle(stream)))


def colour_first_fit(row_ptr, col_idx):
    """The SSOR colouring of a CSR pattern (host numpy arrays): (colour per row, colours)."""
    import numpy as np
    lib = load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    colour = np.empty(max(n, 1), dtype=np.int32)
    nc = c_int32()
    _check(lib.rsolve_colour_first_fit(n, c_void_p(rp.ctypes.data), c_void_p(ci.ctypes.data),
                                       c_void_p(colour.ctypes.data), byref(nc)))
    return colour[:n], nc.value


def gram_tn_noalloc(A, B, stream=None, check=True):
    """gram_tn through rsolve_gram_tn_noalloc (no workspace: the library's static scratch).
    Returns (C, status); C is None when the call failed."""
    import numpy as np
    lib = load()
    p, n = A.shape
    q, n2 = B.shape
    assert n == n2
    C = (c_double * max(p * q, 1))()
    status = lib.rsolve_gram_tn_noalloc(n, c_void_p(A.data_ptr()), n, p, c_void_p(B.data_ptr()), n, q, C,
                                        _stream_handle(stream))
    if check:
        _check(status)
    if status != OK:
        return None, status
    return np.frombuffer(C, dtype=np.float64)[: p * q].reshape(q, p).T.copy(), status


def snapshot_svd(X, k, stream=None):
    """TSQR + Jacobi SVD + basis formation on X given as (c, n) (row c = snapshot c)."""
    import numpy as np
    import torch
    lib = load()
    c, n = X.shape
    ws, nbytes = _kernel_ws(n, c, X.device)
    W = torch.zeros((max(k, 1), n), dtype=torch.float64, device=X.device)
    sig = (c_double * c)()
    ke = c_int32()
    rk = c_int32()
    _check(lib.rsolve_snapshot_svd(n, c_void_p(X.data_ptr()), n, c, k, c_void_p(W.data_ptr()), n, sig, byref(ke),
                                   byref(rk), c_void_p(ws.data_ptr()), nbytes, _stream_handle(stream)))
    return W[: ke.value], np.array(sig[:]), ke.value, rk.value
