"""Build libat.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, binary64 arithmetic without contraction (-ffp-contract=off, so the
evaluation order written in the kernels is the one executed), packed-FP32
instructions disabled for the device code.

Each source is compiled in two passes: the device pass (gfx950 code object,
with the packed-FP32 feature turned off) and the host pass, which embeds that
code object.  The target feature is thereby given only to the compiler that
knows it, instead of also reaching the x86 host pass, which would ignore it
with a warning."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libat.so")
SOURCES = ["at_api.hip", "at_step1d.hip", "at_adj1d.hip", "at_step3d.hip", "at_ws1d.hip",
           "at_util.hip", "at_whole1d.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]
DEVICE_ONLY = ["--offload-device-only", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _run_all(cmds, verbose):
    procs = []
    for cmd, src in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
    bad = [s for p, s in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("hipcc failed for: " + ", ".join(bad))


def build(verbose: bool = False) -> str:
    """Compile every source and link the in-tree libat.so."""
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    dev_cmds, host_cmds, objs = [], [], []
    for src in sources():
        base = os.path.join(objdir, os.path.basename(src))
        fb, obj = base + ".hipfb", base + ".o"
        dev_cmds.append(([HIPCC] + COMMON + DEVICE_ONLY + ["-c", src, "-o", fb], src))
        host_cmds.append(([HIPCC] + COMMON + ["--offload-host-only", "-Xclang",
                                              "-fcuda-include-gpubinary", "-Xclang", fb,
                                              "-c", src, "-o", obj], src))
        objs.append(obj)
    _run_all(dev_cmds, verbose)
    _run_all(host_cmds, verbose)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined"] + objs + [
        "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
