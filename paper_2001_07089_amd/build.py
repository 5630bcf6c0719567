"""Build the HIP library ``_lib/libkamd.so`` for gfx950 with hipcc.

Every kernel translation unit is compiled for gfx950 only, with packed FP32
instructions disabled (``-packed-fp32-ops``); the histogram/MSD unit is also
compiled without floating-point contraction so that its pair distances follow
the definition operation by operation.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUTDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(ROOT, "_build", "kamd")
LIB = os.path.join(OUTDIR, "libkamd.so")
# the compiler's per-kernel resource report (registers, scratch, occupancy)
RESOURCES = os.path.join(ROOT, "_build", "kamd", "kernel_resources.txt")

SOURCES = {
    "kernels_build.hip": [],
    "kernels_force.hip": [],
    "kernels_step.hip": [],
    "kernels_analysis.hip": ["-ffp-contract=off"],
    "static_ws.hip": [],
    "runtime.cpp": [],
}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-pthread", "-Wall", "-Wno-unused-result"]


def _compile(src, extra):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    report = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
    cmd = [hipcc()] + common_flags() + extra + lang + report + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False) -> str:
    """Compile all sources and link ``_lib/libkamd.so``; returns its path."""
    os.makedirs(OUTDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(5, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(_compile, s, e) for s, e in SOURCES.items()]
        objs = []
        report = []
        for f in futs:
            obj, log = f.result()
            objs.append(obj)
            report += [ln for ln in log.splitlines() if "remark:" in ln]
            if verbose and log.strip():
                print("\n".join(ln for ln in log.splitlines() if "remark:" not in ln), file=sys.stderr)
    with open(RESOURCES, "w") as fh:
        fh.write("\n".join(report) + "\n")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
