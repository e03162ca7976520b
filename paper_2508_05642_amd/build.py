"""Build libusp.so (hand-written HIP for gfx950) in-tree with hipcc."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libusp.so")
SRC = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HDR = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [
    os.path.join(os.path.dirname(HERE), "include", "usp.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no hoisting of constant materialisation out of loops: the particle
    # loops inline long math routines whose constants would otherwise stay
    # live in VGPRs for the whole loop
    "-mllvm", "-disable-machine-licm",
    # FP32 divide and sqrt to ~2 ulp (hardware reciprocal/sqrt) instead of
    # the correctly rounded sequences: single precision appears only in the
    # FP32 particle arithmetic, which is held to a tolerance; every discrete
    # decision and all cell quantities are FP64
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
]


def _code(text):
    """The text of a C/C++/HIP source without comments and whitespace (the
    sources hold no string literal with a comment marker in it)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


def fingerprint():
    """SHA-256 of the code of every kernel source and the public header
    (comments and whitespace removed) and the compiler flags: identifies the
    code that a stored counter measurement belongs to."""
    import hashlib
    h = hashlib.sha256()
    for f in SRC + HDR:
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            h.update(_code(fh.read()).encode())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SRC + HDR)


OBJ_DIR = os.path.join(os.path.dirname(HERE), "_build")


def _compile(src):
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    r = subprocess.run(["hipcc"] + flags + ["-c", "-o", obj, src], cwd=HERE,
                       capture_output=True, text=True)
    return obj, r


def build(force=True, verbose=False, jobs=None):
    """Compile every .hip source (one hipcc per source, in parallel) and
    link them into one shared library (always, unless force=False and the
    library is newer than all sources)."""
    if not force and not stale():
        return LIB
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(SRC), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(_compile, SRC))
    for obj, r in res:
        if r.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
        if verbose and r.stderr:
            print(r.stderr)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in res]
    r = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
