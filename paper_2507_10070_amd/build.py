"""Build the gfx950 search library (``libflashann.so``) with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflashann.so")
SOURCES = ["search_kernel.hip", "search_full_u8.hip", "search_full_i8.hip", "search_full_f32.hip",
           "search_pq_u8.hip", "search_pq_i8.hip", "search_pq_f32.hip", "search_pq.hip",
           "api.hip", "agent.cpp", "server.cpp",
           # the graph builder of the input generators, for ann_build_index
           os.path.join("..", "..", "synth", "csrc", "graph_build.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed fp32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    if verbose:
        print(" ".join(cmd))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source into LIB (always recompiles): one object per
    source, compiled in parallel, then linked."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 16)
    tmpdir = tempfile.mkdtemp(prefix="flashann_build_")
    try:
        objs = [os.path.join(tmpdir, "%d_%s.o" % (i, os.path.basename(src)))
                for i, src in enumerate(srcs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda so: _run([HIPCC] + FLAGS + ["-c", so[0], "-o", so[1]], verbose), zip(srcs, objs)))
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC] + FLAGS + ["-shared"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
