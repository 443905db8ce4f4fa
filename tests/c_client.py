"""Build and run the plain-C client of the library (tests/c/abi_client.c).

The client links against the in-tree libstencil.so (found next to it through
a relative run path) and the HIP runtime, and includes only the library's
header and the HIP runtime's C API.
"""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_client.c")
BIN = os.path.join(ROOT, "tests", "c", "abi_client")
PKG = os.path.join(ROOT, "paper_2309_04671_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def compile_client(out: str = BIN) -> str:
    rel = os.path.relpath(PKG, os.path.dirname(os.path.abspath(out)))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror",
           "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
           "-I" + os.path.join(ROOT, "include"), SRC, "-o", out,
           "-L" + PKG, "-lstencil", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/" + rel, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return out


def client_binary(scratch_dir: str) -> str:
    """The client that build() made, or (if it is missing) one compiled now
    into scratch_dir."""
    if os.path.exists(BIN):
        return BIN
    return compile_client(os.path.join(scratch_dir, "abi_client"))


def run_client(*args, binary: str = BIN, timeout: int = 120) -> subprocess.CompletedProcess:
    return subprocess.run([binary] + [str(a) for a in args], capture_output=True, text=True,
                          timeout=timeout)
