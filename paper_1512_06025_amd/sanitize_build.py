"""Host-sanitized build of libbbdg for checking the host code on the CPU.

Builds paper_1512_06025_amd/libbbdg_san.so from the same sources as build.py,
with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(device code is compiled as usual), and with --test runs the CPU test suite
(pytest -m "not gpu") against it: the ASan runtime is preloaded into the
test process and BBDG_LIBRARY points the binding at the sanitized library.
The CPU suite covers the host code of the library: argument validation,
mesh geometry and connectivity, the operator index tables and the dense
nodal operators (built before any device call in bbdg_create), point
location and Bernstein evaluation.

    python paper_1512_06025_amd/sanitize_build.py [--test]
"""
import glob
import os
import subprocess
import sys

from build import ARCH, CSRC, HERE, ROOT, SOURCES, hipcc

LIB = os.path.join(HERE, "libbbdg_san.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")] + HOST_SAN


def asan_runtime():
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        raise RuntimeError("ASan runtime of the ROCm clang not found")
    return rts[-1]


def build():
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".san.o")
        cmd = [hipcc()] + (["-x", "hip"] if src.endswith(".cpp") else []) + FLAGS + [
            "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    rt = asan_runtime()
    # the host objects need the ASan runtime (which carries the UBSan handlers)
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", LIB] + objs + [
        rt, "-Wl,-rpath," + os.path.dirname(rt)]
    subprocess.check_call(cmd)
    for o in objs:
        os.remove(o)
    return LIB


def run_cpu_tests():
    env = dict(os.environ)
    env["BBDG_LIBRARY"] = LIB
    env["LD_PRELOAD"] = asan_runtime() + ((":" + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"  # the HIP runtime keeps its allocations
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.call([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu",
                            "-p", "no:cacheprovider"], env=env, cwd=ROOT)


if __name__ == "__main__":
    print(build(), flush=True)
    if "--test" in sys.argv:
        sys.exit(run_cpu_tests())
