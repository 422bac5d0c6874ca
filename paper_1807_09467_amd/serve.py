"""Serving driver over the rsolve server (include/rsolve_server.h).

`Server` is the ctypes binding (argument marshalling only; the scheduling, batching and every
solve run in the library).  `serving_specs` draws the mixed workload: independent
time-stepping sequences of random degree, mesh, viscosity and length arriving as a Poisson
process; `run_serving` replays it: sequences are admitted by the server's memory budget as
they arrive, each step's system is assembled on the GPU from the sequence's previous solution
and submitted, and every completion is timed from submit to result.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import numpy as np

from . import rsolve
from . import workload as WL

E_BUDGET = -6

SERVER_EXPORTS = ["rsolve_server_create", "rsolve_server_open", "rsolve_server_submit", "rsolve_server_poll",
                  "rsolve_server_close", "rsolve_server_info_get", "rsolve_server_destroy"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool", c_void_p), ("pool_bytes", c_size_t), ("large_workers", c_int32), ("max_batch", c_int32),
                ("max_sequences", c_int32), ("small_fp64", c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", c_uint64), ("seq_id", c_uint64), ("status", c_int32), ("batched", c_int32),
                ("stats", rsolve.Stats), ("t_latency_ms", c_double), ("t_queue_ms", c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("pool_used", c_size_t), ("pool_largest_free", c_size_t), ("sequences", c_int32),
                ("pending", c_int32), ("completed", c_int64), ("batches", c_int64), ("batched_solves", c_int64)]


def _lib():
    lib = rsolve.load()
    if not getattr(lib, "_server_bound", False):
        lib.rsolve_server_create.argtypes = [POINTER(ServerConfig), POINTER(c_void_p)]
        lib.rsolve_server_create.restype = c_int
        lib.rsolve_server_open.argtypes = [c_void_p, POINTER(rsolve.Config), c_int64, c_int64, POINTER(c_uint64)]
        lib.rsolve_server_open.restype = c_int
        lib.rsolve_server_submit.argtypes = [c_void_p, c_uint64, POINTER(rsolve.CSR), c_void_p, c_void_p, c_void_p,
                                             c_double, c_void_p, c_uint64]
        lib.rsolve_server_submit.restype = c_int
        lib.rsolve_server_poll.argtypes = [c_void_p, POINTER(Completion), c_int32, POINTER(c_int32), c_int32]
        lib.rsolve_server_poll.restype = c_int
        lib.rsolve_server_close.argtypes = [c_void_p, c_uint64]
        lib.rsolve_server_close.restype = c_int
        lib.rsolve_server_info_get.argtypes = [c_void_p, POINTER(ServerInfo)]
        lib.rsolve_server_info_get.restype = c_int
        lib.rsolve_server_destroy.argtypes = [c_void_p]
        lib.rsolve_server_destroy.restype = c_int
        lib._server_bound = True
    return lib


class Server:
    """A device memory pool plus worker threads that complete submitted solves asynchronously."""

    def __init__(self, pool_bytes, device=None, large_workers=4, max_batch=256, max_sequences=4096,
                 small_fp64=True):
        import torch
        self.lib = _lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        self.cfg = ServerConfig(self.pool.data_ptr(), int(pool_bytes), large_workers, max_batch, max_sequences,
                                1 if small_fp64 else 0)
        h = c_void_p()
        with torch.cuda.device(self.device):
            rsolve._check(self.lib.rsolve_server_create(byref(self.cfg), byref(h)))
        self.handle = h
        self._cap = 512
        self._buf = (Completion * self._cap)()
        self._keep = {}   # tag -> objects that must outlive the request

    def open(self, n, nnz_max, **cfg):
        """Admit a sequence; returns its id, or None when the pool or the slots are full."""
        import torch
        c = rsolve.make_config(**cfg)
        sid = c_uint64()
        with torch.cuda.device(self.device):
            st = self.lib.rsolve_server_open(self.handle, byref(c), int(n), int(nnz_max), byref(sid))
        if st == E_BUDGET:
            return None
        rsolve._check(st)
        return sid.value

    def submit(self, seq_id, row_ptr, col_idx, val, b, x0, x, tol, ready_event=None, tag=0):
        import torch
        n = int(b.numel())
        A = rsolve.CSR(n, int(val.numel()), rsolve._ptr(row_ptr, torch.int32, n + 1, "row_ptr"),
                       rsolve._ptr(col_idx, torch.int32, None, "col_idx"), rsolve._ptr(val, torch.float64, None, "val"),
                       0, 0)
        ev = ready_event.cuda_event if ready_event is not None else None
        self._keep[tag] = (row_ptr, col_idx, val, b, x0, x, ready_event)
        rsolve._check(self.lib.rsolve_server_submit(
            self.handle, seq_id, byref(A), c_void_p(rsolve._ptr(b, torch.float64, n, "b")),
            c_void_p(rsolve._ptr(x0, torch.float64, n, "x0")), c_void_p(rsolve._ptr(x, torch.float64, n, "x")),
            float(tol), c_void_p(ev), tag))

    def poll(self, timeout_ms=0):
        cnt = c_int32()
        rsolve._check(self.lib.rsolve_server_poll(self.handle, self._buf, self._cap, byref(cnt), int(timeout_ms)))
        out = []
        for i in range(cnt.value):
            c = self._buf[i]
            self._keep.pop(c.tag, None)
            out.append({"tag": c.tag, "seq_id": c.seq_id, "status": c.status, "batched": bool(c.batched),
                        "stats": c.stats.as_dict(), "latency_ms": c.t_latency_ms, "queue_ms": c.t_queue_ms})
        return out

    def close(self, seq_id):
        rsolve._check(self.lib.rsolve_server_close(self.handle, seq_id))

    def info(self):
        i = ServerInfo()
        rsolve._check(self.lib.rsolve_server_info_get(self.handle, byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.rsolve_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


@dataclasses.dataclass
class SeqSpec:
    idx: int
    arrival_s: float
    p: int
    N: int
    eps: float
    steps: int
    seed: int

    def problem(self):
        return WL.Problem(p=self.p, N=self.N, eps=self.eps, dt=5e-3, beta="const")


def serving_specs(nseq=512, rate=200.0, seed=0, degrees=(1, 2, 3), meshes=tuple(range(64, 385, 32)),
                  eps_range=(1e-4, 1e-1), steps_range=(10, 60)):
    """The mixed serving workload: Poisson arrivals at `rate` per second; degree, mesh, log-uniform
    viscosity, length and bump centre drawn per sequence from one seeded generator."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nseq))
    p = rng.choice(np.asarray(degrees), nseq)
    N = rng.choice(np.asarray(meshes), nseq)
    eps = 10.0 ** rng.uniform(np.log10(eps_range[0]), np.log10(eps_range[1]), nseq)
    steps = rng.integers(steps_range[0], steps_range[1] + 1, nseq)
    seeds = rng.integers(0, 2 ** 31 - 1, nseq)
    return [SeqSpec(i, float(arrivals[i]), int(p[i]), int(N[i]), float(eps[i]), int(steps[i]), int(seeds[i]))
            for i in range(nseq)]


class AssemblerCache:
    """One GPU assembler per (degree, mesh); per-sequence variants share its pattern arrays."""

    def __init__(self, device):
        self.device = device
        self.base = {}

    def prepare(self, specs, log=None):
        t0 = time.perf_counter()
        for key in sorted({(s.p, s.N) for s in specs}):
            if key not in self.base:
                prob = WL.Problem(p=key[0], N=key[1], eps=1e-2, dt=5e-3, beta="const")
                asm = WL.Assembler(prob)
                asm.mass_values()
                self.base[key] = WL.GpuAssembler(asm, self.device)
                if log:
                    log(f"pattern Q{key[0]} {key[1]}x{key[1]}: n={asm.pat.n} nnz={asm.pat.nnz}")
        return time.perf_counter() - t0

    def for_spec(self, spec):
        return self.base[(spec.p, spec.N)].variant(spec.problem())


class _Active:
    __slots__ = ("spec", "sid", "gasm", "step", "x", "vals", "b", "ev", "t_assemble")

    def __init__(self, spec, sid, gasm, device):
        import torch
        pat = gasm.asm.pat
        self.spec, self.sid, self.gasm, self.step = spec, sid, gasm, 0
        u0 = torch.from_numpy(WL.initial_condition(spec.problem(), spec.seed)).to(device)
        self.x = [u0, torch.empty_like(u0)]
        self.vals = torch.empty(pat.nnz, dtype=torch.float64, device=device)
        self.b = torch.empty(pat.n, dtype=torch.float64, device=device)
        self.ev = torch.cuda.Event()
        self.t_assemble = 0.0


def run_serving(specs, solver_cfg, tol, device, pool_bytes, large_workers=4, max_batch=256, small_fp64=True,
                cache=None, log=None, keep_solutions=None):
    """Replay `specs` through a new server; returns the per-solve records and a summary.

    keep_solutions: optional set of sequence indices whose solutions are copied out (for the
    alone-versus-mixed comparison)."""
    import torch
    cache = cache or AssemblerCache(device)
    t_gen_setup = cache.prepare(specs, log)
    srv = Server(pool_bytes, device, large_workers=large_workers, max_batch=max_batch, small_fp64=small_fp64)
    stream = torch.cuda.current_stream(device)
    waiting = collections.deque(sorted(specs, key=lambda s: s.arrival_s))
    active = {}
    records = []
    kept = {}
    t_assemble = 0.0
    refused = 0
    tag = 0

    def submit_next(a):
        nonlocal tag, t_assemble
        t0 = time.perf_counter()
        a.gasm.system(a.x[a.step & 1], a.vals, a.b, stream)
        a.ev.record(stream)
        t_assemble += time.perf_counter() - t0
        tag += 1
        srv.submit(a.sid, a.gasm.row_ptr, a.gasm.col_idx, a.vals, a.b, a.x[a.step & 1], a.x[(a.step + 1) & 1],
                   tol, ready_event=a.ev, tag=tag)

    t_start = time.perf_counter()
    t_report = t_start
    while waiting or active:
        if log and time.perf_counter() - t_report > 10.0:
            t_report = time.perf_counter()
            log(f"serving: {len(records)} solves done, {len(active)} sequences active, {len(waiting)} waiting, "
                f"{t_report - t_start:.0f}s")
        now = time.perf_counter() - t_start
        while waiting and waiting[0].arrival_s <= now:
            sp = waiting[0]
            gasm = cache.for_spec(sp)
            pat = gasm.asm.pat
            sid = srv.open(pat.n, pat.nnz, **solver_cfg)
            if sid is None:
                refused += 1
                break
            waiting.popleft()
            a = _Active(sp, sid, gasm, device)
            active[sid] = a
            submit_next(a)
        wait_ms = 2 if active else 0
        if not active and waiting:
            time.sleep(max(0.0, min(0.01, waiting[0].arrival_s - (time.perf_counter() - t_start))))
            continue
        for c in srv.poll(timeout_ms=wait_ms):
            a = active[c["seq_id"]]
            if c["status"] not in (rsolve.OK, rsolve.NOT_CONVERGED):
                raise rsolve.RsolveError(c["status"], f"sequence {a.spec.idx} step {a.step} failed")
            records.append({"seq": a.spec.idx, "step": a.step, "n": a.gasm.asm.pat.n, "latency_ms": c["latency_ms"],
                            "queue_ms": c["queue_ms"], "batched": c["batched"],
                            "iterations": c["stats"]["iterations"], "rel_res": c["stats"]["rel_res_true"],
                            "converged": c["stats"]["converged"]})
            a.step += 1
            if keep_solutions is not None and a.spec.idx in keep_solutions:
                kept.setdefault(a.spec.idx, []).append(a.x[a.step & 1].clone())
            if a.step >= a.spec.steps:
                srv.close(a.sid)
                del active[a.sid]
            else:
                submit_next(a)
    torch.cuda.synchronize(device)
    elapsed = time.perf_counter() - t_start
    info = srv.info()
    srv.destroy()
    lat = np.array([r["latency_ms"] for r in records])
    summary = {
        "solves": len(records),
        "elapsed_s": elapsed,
        "solves_per_s": len(records) / elapsed,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "batched_fraction": float(np.mean([r["batched"] for r in records])),
        "avg_iterations": float(np.mean([r["iterations"] for r in records])),
        "max_rel_residual": float(max(r["rel_res"] for r in records)),
        "all_converged": all(r["converged"] for r in records),
        "batches": info["batches"],
        "mean_batch": info["batched_solves"] / max(info["batches"], 1),
        "admission_refusals": refused,
        "generator_setup_s": t_gen_setup,
        "assembly_s": t_assemble,
    }
    return records, summary, kept
