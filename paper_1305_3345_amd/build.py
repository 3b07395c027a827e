"""Builds libaesgpu.so (HIP kernels for gfx950 plus the C ABI) in the package directory."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libaesgpu.so")
# The LDS gather probe (a stand-alone program the benchmark runs to measure
# the ceiling of the round-table kernels on the machine it runs on).
PROBE_SRC = os.path.join(HERE, "probe", "lds_gather_probe.cpp")
PROBE = os.path.join(HERE, "probe", "lds_gather_probe")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions stay off in every HIP build of this project.
NO_PK_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Per-file instruction-scheduling strategy (LLVM AMDGPU), chosen by measuring
# the tile kernels on 4 KiB pages: see each file's header.
SCHED_FLAGS = {
    "aes_tiles_dec.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compiles every source (always) and links the shared library; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
              f"-I{INCLUDE}", f"-I{CSRC}"] + NO_PK_FP32
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = common + SCHED_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[cmd.index("-c"):cmd.index("-c")] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                            text=True)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[[p.poll() is None for _, p in procs].index(True)][1].wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0]
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln
                 and "warning: unknown target feature" not in ln]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and any(ln.strip() for ln in lines):
            print("\n".join(lines))
    if failed:
        raise RuntimeError("HIP build failed:\n" + "\n\n".join(f"{s}:\n{o}" for s, o in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """Compiles the LDS gather probe (always) and returns its path."""
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17"] + NO_PK_FP32 + [
        "-x", "hip", PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        raise RuntimeError("probe build failed:\n" + out.stdout)
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True))
