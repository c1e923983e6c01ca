"""Build libmsdd.so for gfx950 with hipcc (in-tree, under paper_2106_06404_amd/_build/)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libmsdd.so")

SOURCES = ["band.hip", "band_blocked.hip", "eig.hip", "eig32.hip", "coarse.hip", "dense_blocked.hip", "pcg.hip", "twist.hip", "gmres.hip", "mlp.hip", "msdd.cpp", "net.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def compile_flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result", "-Wno-unused-variable",
        f"-I{os.path.join(ROOT, 'include')}",
        f"-I{CSRC}",
    ]


# Host-code sanitizer build (undefined-behaviour checks on the host planner, the runtime
# around the kernels and the C ABI; device code is built as usual): a separate library
# under _build_ubsan/, loaded instead of the regular one when MSDD_LIB names it.  Any
# undefined behaviour aborts the process with a report.
UBSAN_DIR = os.path.join(HERE, "_build_ubsan")
UBSAN_FLAGS = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
               "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source to an object, then link the shared library (always rebuilds)."""
    out_dir = UBSAN_DIR if sanitize else OUT_DIR
    lib = os.path.join(out_dir, "libmsdd.so")
    extra = UBSAN_FLAGS if sanitize else []
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + compile_flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, txt))
        elif verbose and txt.strip():
            print(txt)
    if failed:
        for src, txt in failed:
            sys.stderr.write(f"--- {src} ---\n{txt}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = lib + f".tmp{os.getpid()}"
    link_extra = []
    if sanitize:
        # the sanitizer runtime is found through the compiler's resource directory
        res = subprocess.check_output([os.path.join(os.path.dirname(os.path.realpath(HIPCC)),
                                                    "..", "lib", "llvm", "bin", "clang++"),
                                       "-print-resource-dir"], text=True).strip()
        rt = os.path.join(res, "lib", "linux")
        link_extra = ["-fsanitize=undefined", "-shared-libsan", f"-Wl,-rpath,{rt}"]
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + link_extra + objs
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--ubsan" in sys.argv))
