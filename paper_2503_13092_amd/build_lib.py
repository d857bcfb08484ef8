"""Builds libds.so (the HIP library behind include/ds.h) for gfx950 with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libds.so")
SOURCES = [os.path.join(HERE, "csrc", "ds_api.hip")]
DEPENDS = SOURCES + [os.path.join(HERE, "csrc", "ds_kernels.h"), os.path.join(ROOT, "include", "ds.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed float32 instructions stay off (never emitted)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print("\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l))
    os.replace(LIB + ".tmp", LIB)
    return LIB


def kernel_source_hash() -> str:
    """Short hash of the kernel sources; ties a stored profile to the code it
    was taken on."""
    import hashlib
    h = hashlib.sha256()
    for p in (os.path.join(HERE, "csrc", "ds_kernels.h"), os.path.join(HERE, "csrc", "ds_api.hip")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPENDS)


if __name__ == "__main__":
    print(build(verbose=True))
