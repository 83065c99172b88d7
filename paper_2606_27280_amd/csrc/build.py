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
           "hn_scan_i8.hip"]
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
        obj = os.path.join(objdir, src + ".o")
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(HERE, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
        if verbose and r.stderr.strip():
            sys.stderr.write(r.stderr)
        return obj

    def check_one(src):
        # device assembly, checked for barriers inside divergent loops
        asm = os.path.join(objdir, src + ".s")
        cmd = ["hipcc", *FLAGS, "-S", "--cuda-device-only", os.path.join(HERE, src), "-o", asm]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc -S failed for %s:\n%s" % (src, r.stderr[-6000:]))
        r = subprocess.run([sys.executable, os.path.join(HERE, "check_barriers.py"), asm, "-v"],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("barrier check failed for %s:\n%s" % (src, r.stdout[-4000:]))
        return asm

    with ThreadPoolExecutor(max_workers=min(8, 2 * len(SOURCES))) as ex:
        futs = [ex.submit(compile_one, s) for s in SOURCES]
        checks = [ex.submit(check_one, s) for s in SOURCES]
        objs = [f.result() for f in futs]
        for c in checks:
            c.result()
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
                           "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
