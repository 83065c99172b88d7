"""Compile libhnsearch.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
SOURCES = ["hn_index.hip", "hn_search.hip", "hn_profile.hip", "hn_scan_f32n.hip",
           "hn_scan_f32w.hip", "hn_scan_bf16.hip", "hn_scan_fp8.hip", "hn_seed.hip",
           "hn_scan_multi.hip", "hn_multi.hip", "hn_layer.hip",
           "hn_scan_i8.hip", "hn_scan_multi_f32.hip", "hn_scan_multi_bf16.hip",
           "hn_scan_multi_fp8.hip", "hn_scan_multi_i8.hip"]
OUT = os.path.join(PKG, "libhnsearch.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA results in ordinary VGPRs: the epilogues read every score, and
         # the accumulation-register form costs one copy instruction per score
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include"), "-I", HERE]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        # one compile per source; -save-temps keeps the device assembly, which
        # is checked for barriers inside divergent loops
        d = os.path.join(objdir, os.path.splitext(src)[0])
        os.makedirs(d, exist_ok=True)
        obj = os.path.join(d, src + ".o")
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(HERE, src), "-o", obj, "-save-temps=obj"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
        if verbose and r.stderr.strip():
            sys.stderr.write(r.stderr)
        asm = os.path.join(d, os.path.splitext(src)[0] + "-hip-amdgcn-amd-amdhsa-gfx950.s")
        if not os.path.exists(asm):
            raise RuntimeError("no device assembly for %s" % src)
        r = subprocess.run([sys.executable, os.path.join(HERE, "check_barriers.py"), asm, "-v"],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("barrier check failed for %s:\n%s" % (src, r.stdout[-4000:]))
        return obj

    # the scan units dominate: start them first
    order = sorted(SOURCES, key=lambda f: not f.startswith("hn_scan"))
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, order))
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
                           "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
