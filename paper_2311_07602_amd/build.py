"""Build ``liblrbg.so`` (the C-ABI library) with hipcc for gfx950.

Always recompiles (the sources in parallel).  Packed-FP32 instructions are disabled in the device code
generator.  The library depends on the HIP runtime by its SONAME
(libamdhip64.so.7), so in a process that has already loaded PyTorch's bundled
copy of the runtime (same SONAME) it binds to that one; standalone it
resolves through its RUNPATH to ROCm's runtime.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblrbg.so")
BUILD = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


SOURCES = ("lrbg_kernels.hip", "lrbg_lrmult.hip", "lrbg_round.hip", "lrbg_short.hip", "lrbg_scratch.hip", "lrbg_add.hip",
           "lrbg_host.cpp")


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one process each) and link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC, *COMMON, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    link_rt = ["-L", os.path.join(ROCM, "lib"), "-lamdhip64"]
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    _run([clang, "-shared", "-fPIC", *objs, "-o", tmp, *link_rt,
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-Wl,--no-undefined", "-lstdc++", "-lm"], verbose)
    os.replace(tmp, LIB)
    return LIB


def sanitizer_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to LD_PRELOAD into a
    process that loads a sanitized library)."""
    import glob
    hits = sorted(glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise FileNotFoundError("no libclang_rt.asan-x86_64.so under " + ROCM)
    return hits[-1]


def build_sanitized(out_dir: str, verbose: bool = False) -> str:
    """The host side of the library (validation, scheduling, layouts) built
    with AddressSanitizer and UndefinedBehaviorSanitizer for CPU tests, linked
    with the device objects of the last build(); returns the library path.
    Only the host code is instrumented: no sanitizer reaches GPU code."""
    os.makedirs(out_dir, exist_ok=True)
    objs = [os.path.join(BUILD, s.rsplit(".", 1)[0] + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError("run build() first; missing " + ", ".join(missing))
    host = os.path.join(out_dir, "lrbg_host_san.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), *san, "-c",
          os.path.join(CSRC, "lrbg_host.cpp"), "-o", host], verbose)
    lib = os.path.join(out_dir, "liblrbg_san.so")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    # the sanitizer runtime is not linked in: the process preloads it
    # (sanitizer_runtime()), which resolves the instrumented object's hooks
    _run([clang, "-shared", "-fPIC", host, *objs, "-o", lib, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lstdc++", "-lm"], verbose)
    return lib


if __name__ == "__main__":
    build(verbose=True)
