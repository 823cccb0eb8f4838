"""Compile libredsea.so (HIP for gfx950 + host C++) in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 only; the objects
are linked into paper_2305_19917_amd/libredsea.so, next to this file.
"""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libredsea.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops off: the compiler must not form packed FP32 instructions.
# Denormals are kept (no flush) so FP32 results follow IEEE semantics.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=fast",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, f))
    return out


def build_id() -> str:
    """First 12 hex digits of the SHA-256 of every source and the header:
    the library reports it in its version string, so timing records can be
    tied to the code that produced them."""
    h = hashlib.sha256()
    for p in sources() + [os.path.join(os.path.dirname(HERE), "include", "redsea.h")]:
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()[:12]


def _compile(src, bid):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ['-DREDSEA_BUILD_ID="%s"' % bid, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    return obj, err


def build(jobs: int = 0) -> str:
    """Compile every source (always) and link libredsea.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    bid = build_id()
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, bid), srcs))
    for _, err in results:
        if err.strip():
            sys.stderr.write(err + "\n")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + [o for o, _ in results]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
