"""Build libqtprod.so (all HIP sources, gfx950) in-tree with hipcc.

Usage:  python -m paper_2212_14318_amd.build [-v] [-i]   (or build() from Python)
        -v prints the commands, -i recompiles only out-of-date sources.

Every translation unit is compiled for gfx950 only, with packed-FP32
instructions disabled, and linked into paper_2212_14318_amd/libqtprod.so.
Object files go to _build/ at the repository root.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(PKG_DIR, "libqtprod.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (install ROCm or set HIPCC)")


def _stale(src: str, obj: str) -> bool:
    """True if obj is missing or older than src or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source and link the shared library; returns its path.

    incremental=True recompiles only sources whose object is out of date.
    """
    os.makedirs(BUILD_DIR, exist_ok=True)
    hipcc = _hipcc()
    procs = []
    objs = []
    sources = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    for src in sources:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and not _stale(os.path.join(CSRC, src), obj):
            continue
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature: harmless noise
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if pr.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = "\n".join(f"--- {s} ---\n{t}" for s, t in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout.decode(errors="replace"))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


# Host-sanitized build of the argument-validation code, for CPU tests of the
# C-ABI: the translation units whose host code validates arguments, carves
# workspaces and builds work lists are compiled with AddressSanitizer and
# UndefinedBehaviorSanitizer on the HOST side only (device code is built as
# usual), then linked with the regular objects of the other units.  The
# result is loaded through QTPROD_LIB with the clang ASan runtime preloaded.
SANITIZED_UNITS = ("api", "batch_host", "noalloc", "tsvd")
SAN_LIB_PATH = os.path.join(BUILD_DIR, "libqtprod_hostsan.so")
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
HOST_SAN_LINK = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -shared-libasan".split()


def asan_runtime() -> str | None:
    """The clang ASan runtime that a host-sanitized library needs preloaded."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_host_sanitized(verbose: bool = False) -> str:
    """Build _build/libqtprod_hostsan.so (needs the regular objects of build())."""
    hipcc = _hipcc()
    sources = sorted(f[:-4] for f in os.listdir(CSRC) if f.endswith(".hip"))
    missing = [u for u in sources if u not in SANITIZED_UNITS and
               not os.path.exists(os.path.join(BUILD_DIR, u + ".o"))]
    if missing:
        raise RuntimeError(f"regular objects missing ({', '.join(missing)}): run build() first")
    procs, objs = [], []
    for u in sources:
        if u not in SANITIZED_UNITS:
            objs.append(os.path.join(BUILD_DIR, u + ".o"))
            continue
        src = os.path.join(CSRC, u + ".hip")
        obj = os.path.join(BUILD_DIR, u + ".hostsan.o")
        objs.append(obj)
        if not _stale(src, obj):
            continue
        cmd = [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument", *HOST_SAN, "-I", os.path.join(ROOT, "include"),
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((u, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for u, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            failed.append((u, out.decode(errors="replace")))
    if failed:
        raise RuntimeError("hipcc (host-sanitized) failed:\n" + "\n".join(f"--- {u} ---\n{t}" for u, t in failed))
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", SAN_LIB_PATH, *objs, *HOST_SAN_LINK]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError("host-sanitized link failed:\n" + res.stdout.decode(errors="replace"))
    return SAN_LIB_PATH


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
    print(path)
