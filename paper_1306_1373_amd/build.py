"""Build the HIP library libdctcodec.so for gfx950 in-tree.

    python -m paper_1306_1373_amd.build [-v]

The result goes to paper_1306_1373_amd/lib/libdctcodec.so.  Packed FP32
instructions are disabled for all device code.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIB_DIR, "libdctcodec.so")
OBJ_DIR = os.path.join(PKG, "_build")
# one object per source, compiled in parallel; the recipe family is spread over
# several sources because its kernel instantiations dominate the build
SOURCES = [os.path.join(CSRC, f) for f in ("api_core.hip", "api_codec.hip", "recipes_n4_n6.hip",
                                           "recipes_n8_n10.hip", "recipes_n12.hip", "api_float.hip",
                                           "api_batch.hip", "api_deblock.hip", "api_probe.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "transform.hpp", "recipe.hpp", "matrix_form.hpp",
                                           "batch.hpp", "deblock.hpp", "staged.hpp", "host.hpp", "rows.hpp",
                                           "codec_launch.hpp")] + [
    os.path.join(INCLUDE, "dctcodec.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
    "-Wall", "-Wextra", "-Wno-unused-parameter",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results straight into VGPRs: no accumulator-register copies
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-fvisibility=hidden",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
LINK_FLAGS = [f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-soname,libdctcodec.so"]


def source_digest() -> str:
    """SHA-256 over the device and host sources of the library: profiles record
    it so that counter figures are only reused for the kernels they measured."""
    import hashlib
    h = hashlib.sha256()
    for path in sorted(SOURCES + HEADERS):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


CODEC_KERNEL_FILES = [os.path.join(CSRC, f) for f in ("kernels.hpp", "transform.hpp", "recipe.hpp", "rows.hpp")]


def codec_kernel_digest() -> str:
    """SHA-256 over what the fused integer codec kernel is compiled from (its
    headers and the compiler flags): a profile of that kernel stays valid while
    this digest is unchanged, whatever else changes in the library."""
    import hashlib
    h = hashlib.sha256()
    for path in CODEC_KERNEL_FILES:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    # include directories by name only: the digest must not depend on where the tree sits
    flags = ["-I" + os.path.basename(f[2:]) if f.startswith("-I") else f for f in FLAGS]
    h.update(" ".join([HIPCC.rsplit("/", 1)[-1], *flags]).encode())
    return h.hexdigest()


def build(verbose: bool = False, extra=None, out: str = LIB, jobs: int = None) -> str:
    """Compile every source to an object (in parallel) and link the library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(os.path.dirname(out), exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(src))[0] + ".o") for src in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = [HIPCC, *FLAGS, *(extra or []), "-c", src, "-o", obj + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(obj + ".tmp", obj)

    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        list(pool.map(compile_one, zip(SOURCES, objs)))
    tmp = out + ".tmp"
    cmd = [HIPCC, *LINK_FLAGS, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
