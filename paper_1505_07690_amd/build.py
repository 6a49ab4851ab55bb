"""Builds libos3d.so in-tree for gfx950 with hipcc.

python -m paper_1505_07690_amd.build   (or paper_1505_07690_amd.build.build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libos3d.so")

SOURCES = ["os3d_api.cpp", "host_setup.cpp", "kernels_bank.hip", "kernels_fft.hip", "kernels_fft4.hip",
           "kernels_plane.hip", "noalloc.hip", "kernels_stream.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    """Compiles every source to an object in a temporary folder (in
    parallel), then links libos3d.so."""
    import concurrent.futures
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    with tempfile.TemporaryDirectory(prefix="os3d_build_") as d:
        def compile_one(src):
            obj = os.path.join(d, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", "-I", CSRC, "-o", obj,
                                                                  os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed compiling {src}")
            return obj
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        cmd = [hipcc] + FLAGS + ["-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libos3d.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
