"""Build libhe.so for gfx950 in-tree (hipcc), one object per source, in parallel.

Usage: python -m paper_2409_16675_amd.build  (or build() from Python).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhe.so")

# longest compiles first: the pool of workers starts them together
SOURCES = ["persistent.hip", "ccmul.hip", "ring_13.hip", "ring_12.hip", "ring_11.hip", "ring_14.hip", "ring_10.hip",
           "kernels.hip", "noalloc.hip", "context.cpp", "plan.cpp", "capi.cpp", "bfv_host.cpp", "batch.cpp", "tune.cpp", "serve.cpp",
           "ccmul.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(ROOT, "include"),
]


def _deps_newer(src, out):
    """True when the object is missing or older than the source or any header."""
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hdrs.append(os.path.join(ROOT, "include", "he.h"))
    return any(os.path.getmtime(f) > t for f in [os.path.join(CSRC, src)] + hdrs)


def _compile(src, incremental=False):
    out = os.path.join(BUILD, src + ".o")
    if incremental and not _deps_newer(src, out):
        return out
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", out]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-8000:]))
    return out


def build(verbose=False, incremental=False):
    """Compile every source (incremental=True skips objects newer than their inputs)."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-8000:])
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


# AddressSanitizer + UndefinedBehaviorSanitizer build of the host sources (the
# device code and its launch glue come from the regular objects), linked as
# _build_san/libhe.so: the host-side tests run against it with the sanitizer
# runtime preloaded (HE_LIBRARY selects it).  Every -fsanitize applies to the
# host pass only.
SAN_BUILD = os.path.join(ROOT, "_build_san")
SAN_LIB = os.path.join(SAN_BUILD, "libhe.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-shared-libasan",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build_sanitized(verbose=False):
    """Link the sanitized library (build() first: the device objects are reused)."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    host = [s for s in SOURCES if s.endswith(".cpp")]
    flags = [f for f in FLAGS if f != "-O3"] + SAN_FLAGS

    def comp(src):
        out = os.path.join(SAN_BUILD, src + ".o")
        r = subprocess.run([HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", out], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc (sanitized) failed for %s:\n%s" % (src, r.stderr[-8000:]))
        return out

    with cf.ThreadPoolExecutor(max_workers=min(8, len(host))) as ex:
        objs = list(ex.map(comp, host))
    objs += [os.path.join(BUILD, s + ".o") for s in SOURCES if not s.endswith(".cpp")]
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stderr[-8000:])
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    if "--sanitized" in sys.argv:
        build_sanitized(verbose=True)
    sys.exit(0)
