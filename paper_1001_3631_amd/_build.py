"""Build the HIP library libteuk.so in-tree for gfx950 (hipcc)."""

import hashlib
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libteuk.so")

SOURCES = ["geometry.cpp", "stencil.hip", "block.hip", "batch_kernel.hip", "adjoint.hip", "static_ws.hip", "flux.hip",
           "capi.cpp", "batch.cpp", "orbit.cpp", "revolve.cpp"]

# -ffp-contract=off: every fused multiply-add is written explicitly, so every
# kernel variant rounds identically.  Packed FP32 instructions are disabled.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def source_hash():
    """Hash of the kernel and library sources; keys the autotuner's cache."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def build(verbose=False, extra_flags=()):
    """Compile every source into libteuk.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + list(extra_flags) + [f'-DTEUK_SOURCE_HASH="{source_hash()}"']
    cmd += ["-I", os.path.join(ROOT, "include"), "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr.strip():
        print(res.stderr, flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
