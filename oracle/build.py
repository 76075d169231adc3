"""Builds the CPU oracle shared library (test infrastructure only).

Plain gcc, binary64 with contraction off so that every product and sum is
rounded as written; binary128 through libquadmath for the per-observation
remainder; OpenMP over particles only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "subsmc_oracle.c")
LIB = os.path.join(HERE, "liboracle_subsmc.so")


SAN_LIB = os.path.join(HERE, "liboracle_subsmc_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize=True builds a copy instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (a CPU check of the oracle's memory accesses and
    arithmetic; load it with libasan preloaded, see run_sanitized_tests)."""
    out = SAN_LIB if sanitize else LIB
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
    cmd = [
        "gcc", "-O2" if not sanitize else "-O1", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
        *(san if sanitize else []),
        "-o", out + ".tmp", SRC, "-lquadmath", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def run_sanitized_tests(pytest_args=("tests", "-q", "-m", "not gpu", "-k", "oracle")) -> int:
    """Runs the oracle's CPU tests against the sanitized build in a child process
    (libasan preloaded, leak detection off: the Python interpreter keeps its
    allocations). Returns the child's exit status."""
    import sys
    build(sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", SUBSMC_ORACLE_LIB=SAN_LIB)
    root = os.path.dirname(HERE)
    return subprocess.run([sys.executable, "-m", "pytest", *pytest_args], cwd=root, env=env).returncode


def ensure_built() -> str:
    alt = os.environ.get("SUBSMC_ORACLE_LIB")
    if alt:
        return alt
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    import sys
    if "--sanitize" in sys.argv:
        sys.exit(run_sanitized_tests())
    print(build(verbose=True))
