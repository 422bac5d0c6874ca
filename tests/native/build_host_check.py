"""Build host_check: the rsolve library sources with AddressSanitizer and UndefinedBehaviorSanitizer
on their host code, linked with the host_check.cpp driver into one executable.

The device code is compiled exactly as for librsolve.so (same flags); the sanitizers are passed with
-Xarch_host so that they instrument the host half only.  Usage:
    python tests/native/build_host_check.py [OUT_DIR]    (default tests/native/_build)
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1807_09467_amd import build as libbuild  # noqa: E402

DEFAULT_OUT = os.path.join(HERE, "_build")
SANITIZE = ["address", "undefined"]


def source_hashes():
    """sha256 of every file the executable is built from (library sources, headers, driver)."""
    files = sorted(glob.glob(os.path.join(libbuild.CSRC, "*.hip")) + glob.glob(os.path.join(libbuild.CSRC, "*.hpp"))
                   + glob.glob(os.path.join(ROOT, "include", "*.h")) + [os.path.join(HERE, "host_check.cpp")])
    out = {}
    for f in files:
        with open(f, "rb") as fh:
            out[os.path.relpath(f, ROOT)] = hashlib.sha256(fh.read()).hexdigest()
    return out


def stale_reason(out_dir: str = DEFAULT_OUT):
    """None when the executable in out_dir was built from the current sources, else why not."""
    exe, manifest = os.path.join(out_dir, "host_check"), os.path.join(out_dir, "host_check.sources.json")
    if not (os.path.exists(exe) and os.path.exists(manifest)):
        return f"{exe} is not built"
    with open(manifest) as fh:
        built = json.load(fh)
    changed = sorted(k for k, v in source_hashes().items() if built.get(k) != v)
    return f"sources changed since the build: {changed}" if changed else None


def host_sanitizer_flags():
    out = ["-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    for s in SANITIZE:
        out += ["-Xarch_host", f"-fsanitize={s}"]
    return out


def build(out_dir: str = DEFAULT_OUT) -> str:
    obj_dir = os.path.join(out_dir, "obj")
    os.makedirs(obj_dir, exist_ok=True)
    cc = libbuild.hipcc()
    hashes = source_hashes()        # taken before compiling: an edit during the build marks it stale
    base = [*libbuild.flags(), *host_sanitizer_flags()]

    def compile_one(src):
        obj = os.path.join(obj_dir, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        r = subprocess.run([cc, *base, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    srcs = [os.path.join(libbuild.CSRC, s) for s in libbuild.SOURCES] + [os.path.join(HERE, "host_check.cpp")]
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = os.path.join(out_dir, "host_check")
    # the link step names no device source, so the runtime flags go to the host link directly
    link = [cc, f"--offload-arch={libbuild.ARCH}", *[f"-fsanitize={s}" for s in SANITIZE], "-fno-gpu-sanitize",
            "-o", exe + ".tmp", *objs]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(exe + ".tmp", exe)
    with open(os.path.join(out_dir, "host_check.sources.json"), "w") as fh:
        json.dump(hashes, fh, indent=0, sort_keys=True)
    return exe


def run_env():
    """Environment for running host_check: leak checking off (the HIP runtime keeps allocations
    until exit), every UBSan finding fatal, reports with a stack trace."""
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else DEFAULT_OUT))
