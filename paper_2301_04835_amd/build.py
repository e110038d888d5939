"""Build libsampx.so (hand-written HIP for gfx950) in-tree with hipcc.

Every source under csrc/ is compiled to an object in _build/ (in parallel)
and linked into paper_2301_04835_amd/libsampx.so; the sources under
measure/ (kernel timing and bandwidth probes for benchmarks) into
libsampx_measure.so, which links libsampx.so.  Packed FP32 instructions
are switched off for the device code; the host pass warns that it does not
know that target feature, which is harmless.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
MSRC = os.path.join(HERE, "measure")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsampx.so")
MLIB = os.path.join(HERE, "libsampx_measure.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
         "-Wno-unused-command-line-argument"]


def sources(d=CSRC):
    return sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith((".hip", ".cpp")))


def _warnings(text):
    """Compiler warnings other than the host pass's note about the packed-FP32
    target feature (expected: the flag is meant for the device code)."""
    return [l for l in text.splitlines() if "warning:" in l and "packed-fp32-ops" not in l]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(os.path.dirname(src)) + "_" + os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))
    for w in _warnings(r.stderr):
        print(w, file=sys.stderr)
    return obj


def _link(objs, out, extra=()):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + list(extra) + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs, msrcs = sources(CSRC), sources(MSRC)
    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_compile, srcs + msrcs))
    _link(objs[:len(srcs)], LIB)
    _link(objs[len(srcs):], MLIB, ["-L" + HERE, "-lsampx", "-Wl,-rpath,$ORIGIN"])
    if verbose:
        print("built", LIB, "and", MLIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
