"""Build libpa.so (gfx950 HIP kernels + host runtime) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpa.so")

SOURCES = ["pa_kernels.hip", "pa_mlp.hip", "pa_noalloc.hip", "pa_host.cpp", "pa_planner.cpp", "pa_plan.cpp", "pa_batch.cpp",
           "pa_model.cpp", "pa_tune.cpp"]
HEADERS = ["pa_internal.h", "pa_plan.h", "pa_mlp.h"]

# -ffp-contract=off: no implicit FMA anywhere (the FP64 corner values are a
# fixed sequence of explicit fma); packed FP32 instructions are disabled.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _scratch_kernels(remarks: str):
    """(kernel, bytes per lane) of every kernel whose resource-usage remark
    reports private (scratch) memory.  The kernels are written to need none:
    register spills to scratch are treated as a build error."""
    out, name = [], None
    for line in remarks.splitlines():
        if "Function Name: " in line:
            name = line.split("Function Name: ", 1)[1].split()[0]
        elif "ScratchSize [bytes/lane]: " in line and name:
            n = int(line.split("ScratchSize [bytes/lane]: ", 1)[1].split()[0])
            if n > 0:
                out.append((name, n))
    return out


def _newest_input():
    paths = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "pa.h"), __file__]
    return max(os.path.getmtime(p) for p in paths)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= _newest_input():
        return LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = ["hipcc", "-x", "hip"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        out = p.communicate()[0].decode()
        scratch = _scratch_kernels(out)
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                 and not l.lstrip().startswith(("|", "^")) and not l.rstrip().endswith(":")]
        if scratch:
            lines.append("kernels using scratch memory: " + ", ".join(f"{k} ({n} B/lane)" for k, n in scratch))
        if p.returncode != 0 or scratch or (verbose and lines):
            sys.stderr.write(" ".join(cmd) + "\n" + "\n".join(lines) + "\n")
        failed |= p.returncode != 0 or bool(scratch)
    if failed:
        raise RuntimeError("libpa build failed")
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
