"""Build the HIP/C++ library ``libftlm.so`` in-tree for gfx950.

Every source under ``csrc/`` is compiled by hipcc (device code for gfx950 only)
into ``_build/`` and linked into ``paper_2607_17429_amd/libftlm.so``.  Packed
FP32 vector instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(HERE, "libftlm.so")
ARCH = os.environ.get("FTLM_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Wno-unknown-cuda-version",
]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc()] + COMMON + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [_hipcc()] + COMMON + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _stale(src: str, newest_header: float) -> bool:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    return os.path.getmtime(obj) < max(os.path.getmtime(src), newest_header)


def build(jobs: int | None = None, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those older than their
    object file or any header) and link libftlm.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    newest = max(os.path.getmtime(h) for h in headers)
    todo = [x for x in srcs if _stale(x, newest)] if incremental else srcs
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD, os.path.basename(x) + ".o") for x in srcs]
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources ({len(todo)} compiled)", file=sys.stderr)
    return OUT


# host-only sources: groups and irreps, Ritz data and thermal sums, their C entry points
HOST_ONLY = ("group.cpp", "thermo.cpp", "tune_cache.cpp", "capi_host.cpp")


SANITIZERS = {"address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
              "thread": ["-fsanitize=thread"]}


def build_host_sanitized(out_dir: str | None = None, verbose: bool = False, kind: str = "address") -> str:
    """The host-only part of the library (HOST_ONLY) built by g++ with the
    address and undefined-behaviour sanitizers (kind "address") or the
    thread sanitizer (kind "thread"), HIP headers for declarations only (no
    device code), as ``libftlm_host_<kind>.so`` in out_dir (default
    _build/sanitize).  Load it with the sanitizer runtime preloaded (see
    sanitizer_env) and FTLM_LIBRARY pointing at it."""
    out_dir = out_dir or os.path.join(BUILD, "sanitize", kind)
    os.makedirs(out_dir, exist_ok=True)
    san = SANITIZERS[kind]
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-fno-omit-frame-pointer"] + san + [
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = []
    for f in HOST_ONLY:
        obj = os.path.join(out_dir, f + ".o")
        cmd = ["g++"] + flags + ["-c", os.path.join(CSRC, f), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        objs.append(obj)
    out = os.path.join(out_dir, f"libftlm_host_{kind}.so")
    cmd = ["g++", "-shared", "-pthread", san[0], "-Wl,-z,defs", "-o", out] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {out}", file=sys.stderr)
    return out


def sanitizer_env(lib_path: str, kind: str = "address") -> dict:
    """Environment for a Python process that loads the sanitized host library:
    the sanitizer runtime preloaded (Python itself is not instrumented), leak
    checking off (the interpreter keeps its allocations), every finding fatal."""
    def lib_of(name):
        return subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()

    env = dict(os.environ)
    # libstdc++ right behind the runtime, so that ASan finds the C++ runtime's
    # functions it intercepts (exceptions) when it starts
    runtime = "libasan.so" if kind == "address" else "libtsan.so"
    env["LD_PRELOAD"] = lib_of(runtime) + ":" + lib_of("libstdc++.so")
    env["FTLM_LIBRARY"] = lib_path
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:alloc_dealloc_mismatch=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:report_signal_unsafe=0"
    return env


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
