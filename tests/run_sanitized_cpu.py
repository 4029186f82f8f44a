#!/usr/bin/env python
"""Run the CPU test suite (-m "not gpu") against sanitized builds.

The oracle (oracle/liboracle_sanitized.so) and the host half of the library
(paper_2608_08287_amd/variants/libtsdf_sanitized.so: argument checks, layout
and workspace arithmetic, the region allocator, server parameter checks) are
built with AddressSanitizer and UndefinedBehaviorSanitizer by ROCm's clang,
whose ASan runtime is preloaded into the test process (Python itself is not
instrumented, so the runtime must be loaded first).  Any report ends the run
with a non-zero status.  Leak detection is off: the interpreter and torch keep
memory until exit by design.

    python tests/run_sanitized_cpu.py            # build both, then run
    python tests/run_sanitized_cpu.py --no-build # run against existing builds
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def asan_runtime() -> str:
    from oracle import build as orabuild
    r = subprocess.run([orabuild.CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError(f"no ASan runtime next to {orabuild.CLANGXX}")
    return path


def main() -> int:
    from oracle import build as orabuild
    from paper_2608_08287_amd import build as libbuild

    if "--no-build" not in sys.argv:
        orabuild.build(verbose=True, sanitize=True)
        libbuild.build(variant="sanitized")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:"
                        "detect_odr_violation=0:new_delete_type_mismatch=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "TSDF_LIBRARY": libbuild.variant_path("sanitized"),
        "ORACLE_LIBRARY": orabuild.SANITIZED_OUT,
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x",
           "-q"] + [a for a in sys.argv[1:] if a != "--no-build"]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main())
