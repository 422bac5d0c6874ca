"""SpMV shape autotuner with a JSON cache.

On first use for a (device, precision, n, nnz) the sequence's Arnoldi product is timed for
every shape the library offers (rsolve_tune_spmv: storage format x lanes per row x entries per
lane x block order, HIP events on the sequence's own buffers) and the fastest is stored; later sequences of
the same size reuse it without timing.  The kernel work and its timing run in the library;
this module only keys, stores and applies the result.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "rsolve",
                             "spmv_shapes.json")


def _key(seq, nnz):
    import torch
    name = torch.cuda.get_device_name(seq.device)
    prec = "fp32" if seq.cfg.precision == 1 else "fp64"
    return f"{name}|{prec}|n={seq.n}|nnz={nnz}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_sequence(seq, row_ptr, col_idx, val, cache_path=DEFAULT_CACHE, reps=20, retune=False):
    """Apply the fastest Arnoldi SpMV shape for this sequence's matrix size, timing it if the cache
    has no entry (or retune).  Returns (shape dict, source: "cache" or "timed", all timings)."""
    key = _key(seq, int(val.numel()))
    table = _load(cache_path) if cache_path else {}
    if key in table and not retune:
        sh = table[key]
        seq.set_spmv_shape(sh["lanes_per_row"], sh["vec"], sh["xcd_remap"], sh.get("format", "csr"))
        return sh, "cache", []
    t0 = time.perf_counter()
    res = seq.tune_spmv(row_ptr, col_idx, val, reps=reps)
    best = dict(res[0])
    best["tuned_in_s"] = time.perf_counter() - t0
    default = seq.spmv_shape()
    fields = ("format", "lanes_per_row", "vec", "xcd_remap")
    match = [r for r in res if all(r[f] == default[f] for f in fields)]
    best["default_us"] = match[0]["us"] if match else None
    seq.set_spmv_shape(best["lanes_per_row"], best["vec"], best["xcd_remap"], best["format"])
    if cache_path:
        table = _load(cache_path)
        table[key] = best
        _store(cache_path, table)
    return best, "timed", res
