"""Build libttfv.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2408_03483_amd.build      (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libttfv.so")
SOURCES = ["kernels.hip", "gemm.hip", "tsqr.hip", "cholqr.hip", "jacobi.hip", "cross.hip", "tt_ops.hip",
           "fixed.hip", "fv.hip", "grid.hip", "tt_nd.hip", "mlp.hip", "capi.hip", "stencils.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objs = []
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS[:-3] + ["-c"] + lang + [os.path.join(CSRC, src), "-o", obj]
        cmd = [c for c in cmd if c != "-shared"]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT)))
    failed = False
    for src, cmd, p in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 target feature: harmless
        lines = [l for l in txt.splitlines() if "packed-fp32-ops" not in l]
        if p.returncode != 0:
            failed = True
            print(f"[build] {src} FAILED\n" + "\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc compilation failed")
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
