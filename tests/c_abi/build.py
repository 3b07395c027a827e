"""Builds tests/c_abi/abi_client: a C-ABI client of libaesgpu.so checked
against the oracle (test infrastructure; needs both libraries built)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "abi_client.cpp")
EXE = os.path.join(HERE, "abi_client")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    """Compiles the client (always) and returns its path."""
    lib_dir = os.path.join(ROOT, "paper_1305_3345_amd")
    oracle_dir = os.path.join(ROOT, "oracle")
    tmp = EXE + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", tmp,
           f"-L{lib_dir}", "-laesgpu", f"-L{oracle_dir}", "-loracle",
           "-Wl,-rpath,$ORIGIN/../../paper_1305_3345_amd", "-Wl,-rpath,$ORIGIN/../../oracle"]
    if verbose:
        print(" ".join(cmd))
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode:
        raise RuntimeError("abi_client build failed:\n" + out.stderr)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
