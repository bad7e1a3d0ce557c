"""Build step of the HIP library ``libpond.so`` for gfx950 (MI355X).

hipcc compiles the kernels and the C-ABI host code into one shared library next
to this file.  Packed-FP32 instructions are disabled for all device code; hipcc's
host pass warns that it does not know that target feature, which is harmless.

Floating-point contraction is limited to single source expressions
(-ffp-contract=on): a multiply-add is fused the same way wherever the per-node
code is inlined, so every kernel variant (HBM gather, each tile shape, the
batched kernel) produces the same bits.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpond.so")
SOURCES = ["pond_kernels.hip", "pond_kernels25.hip", "pond_batch.hip", "pond_server.hip",
           "pond_api.hip", "pond_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose: bool = False, jobs: int = 2, defines=(), out: str = LIB) -> str:
    """Compile libpond.so (always recompiles) and return its path.  ``defines``
    are extra -D compile-time tuning macros; ``out`` the library path."""
    tmp = out + ".tmp"
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *["-D" + d for d in defines], "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
