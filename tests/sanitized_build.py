"""Host AddressSanitizer + UndefinedBehaviorSanitizer build of libslrx, for running
the CPU ABI tests against instrumented host code.  The device code is compiled as
in the product build; only the host side is instrumented (hipcc's -Xarch_host
before each sanitizer option).  Output: _build/hostsan/libslrx.so, rebuilt when a
source or header is newer than it.  Test infrastructure only."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

from paper_1704_04511_amd import build as product

OUT = os.path.join(product.ROOT, "_build", "hostsan")
LIB = os.path.join(OUT, "libslrx.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def runtime() -> str:
    """The clang AddressSanitizer runtime the instrumented library needs preloaded."""
    pat = os.path.join(product.rocm_path(), "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                       "libclang_rt.asan-x86_64.so")
    found = sorted(glob.glob(pat))
    if not found:
        raise FileNotFoundError(pat)
    return found[-1]


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    srcs = glob.glob(os.path.join(product.CSRC, "*")) + glob.glob(os.path.join(product.ROOT, "include", "*.h"))
    return max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(LIB)


def build() -> str:
    if not _stale():
        return LIB
    hipcc = shutil.which("hipcc") or os.path.join(product.rocm_path(), "bin", "hipcc")
    os.makedirs(OUT, exist_ok=True)
    objs, jobs = [], []
    for src in product.SOURCES:
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        objs.append(obj)
        jobs.append([hipcc, *product.HIPCC_FLAGS, *HOST_SAN, "-c", os.path.join(product.CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(product._run, jobs))
    tlib = product.torch_lib_dir()
    rlib = os.path.join(product.rocm_path(), "lib")
    clang = os.path.join(product.rocm_path(), "lib", "llvm", "bin", "clang++")
    tmp = LIB + ".tmp"
    product._run([clang, "-shared", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp, *objs,
                  "-L", tlib, "-l:libamdhip64.so", "-l:librocsolver.so", "-l:librocblas.so",
                  "-L", rlib, "-l:librocprofiler-sdk-roctx.so",
                  f"-Wl,-rpath,{tlib}", f"-Wl,-rpath,{rlib}", "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
