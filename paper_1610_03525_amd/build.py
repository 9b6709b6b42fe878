"""Build libptg.so (HIP, gfx950) in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, with packed-FP32 code generation
disabled, and linked into one shared library whose exported symbols are the C ABI in
include/ptg.h.
"""
import os
import subprocess
import sys
import glob

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libptg.so")
LOADGEN = os.path.join(HERE, "libptg_loadgen.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep matrix-core accumulators in ordinary VGPRs: the same registers are also updated
    # by VALU code, and AGPR<->VGPR copies around every MFMA cost more than they save
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_loadgen(verbose)
    return LIB


def build_loadgen(verbose: bool = False) -> str:
    """libptg_loadgen.so: the native open-loop stream driver used by the serving benchmark
    (host code over libptg's C ABI, found next to it at run time)."""
    src = os.path.join(HERE, "loadgen", "ptg_loadgen.cpp")
    cmd = [HIPCC] + FLAGS + ["-I" + os.path.join(HERE, "loadgen"), "-shared", src, "-L" + HERE, "-lptg",
                             "-Wl,-rpath,$ORIGIN", "-lpthread", "-o", LOADGEN + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed (loadgen):\n" + p.stdout.decode(errors="replace"))
    os.replace(LOADGEN + ".tmp", LOADGEN)
    return LOADGEN


def _drain(procs):
    errors = []
    while procs:
        src, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            errors.append(f"{src}:\n{text}")
        elif text.strip():
            # keep warnings visible (the host pass warns about the packed-fp32 feature flag)
            lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if lines:
                print("\n".join(lines), file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
