"""Build libbeadscf.so for gfx950 in-tree.

Steps: run csrc/gen_eri.py into csrc/generated/, compile every .hip/.cpp
translation unit with hipcc (in parallel), link the shared library next to
this file.  ``python -m paper_1601_02713_amd.build [--force]``.
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "generated")
OBJ = os.path.join(os.path.dirname(HERE), "_build", "obj")
LIB = os.path.join(HERE, "libbeadscf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPFLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", CSRC, "-I", GEN, "-I", os.path.join(ROCM, "include"),
]


def _sources():
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")) +
                  glob.glob(os.path.join(GEN, "*.hip")))
    return srcs


_INC = re.compile(r'^\s*#\s*include\s*"([^"]+)"', re.M)


def _deps_mtime(path, seen=None):
    """Newest mtime of a file and of every quoted include it pulls in."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return 0.0
    seen.add(path)
    t = os.path.getmtime(path)
    with open(path, errors="replace") as f:
        text = f.read()
    for inc in _INC.findall(text):
        for d in (os.path.dirname(path), CSRC, GEN):
            cand = os.path.normpath(os.path.join(d, inc))
            if os.path.exists(cand):
                t = max(t, _deps_mtime(cand, seen))
                break
    return t


def _compile(src, force, hdr_time=None):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not force and os.path.exists(obj):
        if os.path.getmtime(obj) > _deps_mtime(src):
            return obj, None
    cmd = ["hipcc"] + HIPFLAGS + ["-Rpass-analysis=kernel-resource-usage", "-x", "hip", "-c", src,
                                  "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return obj, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    # per-kernel resource usage (VGPRs, scratch bytes per lane) for inspection
    with open(obj + ".resources.txt", "w") as f:
        for ln in r.stderr.splitlines():
            if "remark:" in ln and any(k in ln for k in ("Function Name", "VGPRs:", "AGPRs:",
                                                          "ScratchSize", "Occupancy", "LDS Size")):
                f.write(ln.split("remark:", 1)[1].replace(" [-Rpass-analysis=kernel-resource-usage]", "") + "\n")
    os.replace(obj + ".tmp", obj)
    return obj, None


def build(force: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    gen_script = os.path.join(CSRC, "gen_eri.py")
    stamp = os.path.join(GEN, "classes.h")
    if force or not os.path.exists(stamp) or os.path.getmtime(stamp) < os.path.getmtime(gen_script):
        subprocess.check_call([sys.executable, gen_script, GEN])
    srcs = _sources()
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs, errs = [], []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, err in ex.map(lambda s: _compile(s, force), srcs):
            objs.append(obj)
            if err:
                errs.append(err)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(errs))
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs):
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
            "-L", os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas", "-lamdhip64",
            f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host sanitizer variant (a test build, not the product): the host side of
# engine.cpp instrumented with AddressSanitizer and UndefinedBehaviorSanitizer,
# device code unchanged, linked with the other objects into
# _san/libbeadscf_san.so, plus the C-ABI driver tests/native/engine_san_main.c
# (the sanitizer runtimes come with the executable).
SAN_DIR = os.path.join(HERE, "_san")
SAN_FLAGS = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build_host_sanitized() -> str:
    build(verbose=False)
    os.makedirs(SAN_DIR, exist_ok=True)
    eng = os.path.join(CSRC, "engine.cpp")
    obj = os.path.join(SAN_DIR, "engine.cpp.o")
    host_only = [a for f in SAN_FLAGS for a in ("-Xarch_host", f)]
    subprocess.check_call(["hipcc"] + HIPFLAGS + host_only + ["-x", "hip", "-c", eng, "-o", obj])
    objs = [o if os.path.basename(o) != "engine.cpp.o" else obj
            for o in (os.path.join(OBJ, os.path.basename(s) + ".o") for s in _sources())]
    lib = os.path.join(SAN_DIR, "libbeadscf_san.so")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + objs + [
        "-L", os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas", "-lamdhip64",
        f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"])
    exe = os.path.join(SAN_DIR, "engine_san")
    root = os.path.dirname(HERE)
    clangxx = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
    subprocess.check_call([clangxx] + SAN_FLAGS + [
        "-I", os.path.join(root, "include"), "-x", "c",
        os.path.join(root, "tests", "native", "engine_san_main.c"),
        "-L", SAN_DIR, "-lbeadscf_san", "-Wl,-rpath,$ORIGIN", "-o", exe])
    print(f"built {exe}")
    return exe


if __name__ == "__main__":
    if "--host-sanitize" in sys.argv:
        build_host_sanitized()
    else:
        build(force="--force" in sys.argv)
