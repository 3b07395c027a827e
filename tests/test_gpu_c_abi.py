"""The library used from C alone: tests/c_abi/abi_client (include/aesgpu.h,
hipMalloc buffers, no Python or torch in the process) runs the mixed batch,
the single-op calls, a plan and its graph, the persistent serving engine and
the host route's batch, and checks each against the oracle byte for byte.
Run as a child process; it prints one "c abi ok" line on success."""
import importlib.util
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c_abi_client():
    exe = os.path.join(HERE, "c_abi", "abi_client")
    if not os.path.exists(exe):  # normally built by __graft_entry__.build()
        spec = importlib.util.spec_from_file_location(
            "c_abi_build", os.path.join(HERE, "c_abi", "build.py"))
        client_build = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(client_build)
        client_build.build()
    print("\n[gpu] C ABI client", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr, flush=True)
    assert out.returncode == 0, out.stderr
    assert "c abi ok" in out.stdout
