"""Build ``libtsdf.so`` (HIP for gfx950) in-tree with hipcc.

Compile flags that the kernels rely on:
  -ffp-contract=off     the band walk must round every float32 operation
                        separately (no FMA) so voxel choices are exact;
  -munsafe-fp-atomics   float atomic adds become the hardware instruction
                        instead of a compare-exchange loop (the pool lives in
                        ordinary device memory, where that instruction is exact);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                        no packed fp32 math is generated.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtsdf.so")
SOURCES = ([os.path.join(CSRC, n) for n in ("tsdf_api.cpp", "tsdf_batch.cpp", "tsdf_arena.cpp",
                                             "tsdf_server.cpp", "tsdf_kernels.hip", "tsdf_mesh.hip")]
           + sorted(glob.glob(os.path.join(CSRC, "tsdf_fuse_k*.hip"))))
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]


# Libraries built with one design alternative switched on, for measuring it
# against the shipped choice (the switches are described in tsdf_device.h).
# They load in place of libtsdf.so when TSDF_LIBRARY names them.
VARIANTS = {
    "first_read_coherent": ["-DTSDF_FIRST_READ_COHERENT=1"],
    "keyset_ballot": ["-DTSDF_KEYSET_BALLOT=1"],
    # the host half under AddressSanitizer and UndefinedBehaviorSanitizer (the
    # device code is built as shipped); the sanitizer runtime comes from the
    # process that loads the library (tests/run_sanitized_cpu.py preloads it)
    "sanitized": ["-g", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined"],
}
VARIANT_DIR = os.path.join(HERE, "variants")


def variant_path(name: str) -> str:
    return os.path.join(VARIANT_DIR, f"libtsdf_{name}.so")


def build(verbose: bool = False, extra=(), jobs: int = 0, variant: str = "") -> str:
    """Compile every translation unit in parallel, then link libtsdf.so (or,
    with `variant`, the library of that design alternative)."""
    extra = list(extra) + (VARIANTS[variant] if variant else [])
    out = variant_path(variant) if variant else OUT
    build_dir = BUILD_DIR + (f"_{variant}" if variant else "")
    os.makedirs(build_dir, exist_ok=True)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)

    def compile_one(src):
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        # the host pass does not know the device-only feature: drop that one line
        err = "".join(line for line in r.stderr.splitlines(keepends=True)
                      if "'-packed-fp32-ops' is not a recognized feature" not in line)
        if err:
            print(err, end="", file=sys.stderr, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("-v", action="store_true", help="print the commands")
    ap.add_argument("--variant", choices=sorted(VARIANTS), default="",
                    help="build the library of one design alternative instead")
    a = ap.parse_args()
    print(build(verbose=a.v, variant=a.variant))
