"""Build the simulator library's own sources for the host, with the HIP emulation of
tests/emu/hip/hip_runtime.h, under AddressSanitizer and UndefinedBehaviorSanitizer.

The kernel sources are compiled as they are, with one textual change: a dynamically sized LDS
array (`extern __shared__ T name[];`) becomes a pointer to the workgroup's emulated LDS block.
The result, tests/emu/_build/libeulerq_emu.so, exports the same C ABI as libeulerq.so; it must
be loaded into a process that has the ASan runtime preloaded (see `asan_env`).
"""
import fcntl
import hashlib
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2402_13259_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libeulerq_emu.so")
KERNEL_SOURCES = ["eq_kernels.hip", "eq_grad.hip", "eq_peak.hip", "eq_sojourn.hip", "eq_capi.cpp"]
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-pthread",
         "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-ffp-contract=off", "-fno-fast-math", "-Wno-unknown-pragmas"]
DYN_LDS = re.compile(r"extern\s+__shared__\s+(\w+)\s+(\w+)\s*\[\s*\]\s*;")


def _sources():
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h", ".cpp")))
    return [os.path.join(CSRC, f) for f in files] + [os.path.join(HERE, "hipemu.cpp"),
                                                   os.path.join(HERE, "hip", "hip_runtime.h"),
                                                   os.path.join(ROOT, "include", "eulerq.h")]


def _stamp() -> str:
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for p in _sources():
        h.update(p.encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def build(force: bool = False) -> str:
    """Compile (if the sources changed) and return the path of the emulated library.  Processes
    that call this together (parallel test workers) build one at a time; the later ones find the
    library current."""
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        return _build_locked(force)


def _build_locked(force: bool) -> str:
    stamp_path = os.path.join(OUT, "stamp")
    stamp = _stamp()
    if not force and os.path.exists(LIB) and os.path.exists(stamp_path) and open(stamp_path).read() == stamp:
        return LIB
    src_dir = os.path.join(OUT, "src")
    os.makedirs(src_dir, exist_ok=True)
    for f in os.listdir(CSRC):
        if f.endswith((".hip", ".h", ".cpp")):
            text = open(os.path.join(CSRC, f)).read()
            text = DYN_LDS.sub(r"\1 *\2 = (\1 *)::emu::dyn_lds();", text)
            with open(os.path.join(src_dir, f), "w") as fh:
                fh.write(text)
    inc = ["-I", HERE, "-I", src_dir, "-I", os.path.join(ROOT, "include")]
    units = [os.path.join(src_dir, f) for f in KERNEL_SOURCES] + [os.path.join(HERE, "hipemu.cpp")]

    def compile_one(path):
        obj = os.path.join(OUT, os.path.basename(path) + ".o")
        subprocess.run(["g++", *FLAGS, *inc, "-x", "c++", "-c", path, "-o", obj], check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, units))
    tmp = LIB + ".tmp"
    subprocess.run(["g++", *FLAGS, "-shared", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    with open(stamp_path, "w") as fh:
        fh.write(stamp)
    return LIB


def asan_env() -> dict:
    """Environment for a child process that loads the emulated library: the GCC ASan runtime
    preloaded, leak checks off (the Python interpreter keeps its own allocations)."""
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


if __name__ == "__main__":
    print(build(force=True))
