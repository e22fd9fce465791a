"""Build ``libotip.so`` (all HIP sources for gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libotip.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("OTIP_ARCH", "gfx950")

# -packed-fp32-ops: no packed FP32 instructions in any HIP code
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]
# per-source additions (none at present)
FILE_FLAGS = {}


def sources():
    return sorted(os.path.join(SRC, f) for f in os.listdir(SRC)
                  if f.endswith((".hip", ".cpp")))


def source_id() -> str:
    """Hash of every library source and the ABI header: compiled into the
    library (otip_source_id) and compared by the binding at load time, so a
    library built from other sources is refused instead of silently used."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(SRC) if f.endswith((".hip", ".cpp", ".h")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(SRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(HERE, "..", "include", "otip.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    deps = [src] + [os.path.join(SRC, h) for h in os.listdir(SRC) if h.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "otip.h"))
    extra = []
    if os.path.basename(src) == "api.hip":
        # carries the source hash: rebuilt whenever any source changes
        deps += sources()
        extra = [f'-DOTIP_SOURCE_ID="{source_id()}"']
    if os.path.exists(obj) and all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps):
        return obj, ""
    cmd = (["hipcc"] + HIPFLAGS + FILE_FLAGS.get(os.path.basename(src), []) + extra +
           ["-c", src, "-o", obj])
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msg}")
    return obj, msg


def build(force: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    if force:
        for f in os.listdir(OBJ):
            os.remove(os.path.join(OBJ, f))
    srcs = sources()
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = [o for o, _ in ex.map(_compile, srcs)]
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
