"""Every kernel of the built library is defined in exactly one translation
unit.  A kernel template instantiated in two units gets two device copies
behind one host launch stub, and which copy a launch runs is then up to the
runtime's registration order; with identical sources that is harmless, but it
hides any difference between the units' builds.  The check reads the symbol
tables of the objects the build leaves in _build/ (skipped before a build)."""
import glob
import re
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_each_kernel_stub_defined_in_one_object():
    objs = sorted(glob.glob(os.path.join(ROOT, "_build", "*", "*.hip.o")))
    nm = shutil.which("nm")
    if not objs or nm is None:
        pytest.skip("no built objects (run the build first)")
    where = {}
    for o in objs:
        out = subprocess.run([nm, "--defined-only", o], capture_output=True, text=True,
                             check=True).stdout
        for line in out.splitlines():
            parts = line.split()
            if len(parts) == 3 and parts[1] in "TW" and "__device_stub__" in parts[2]:
                where.setdefault(parts[2], []).append(os.path.basename(o))
    assert where, "no kernel launch stubs found"
    dup = {k: v for k, v in where.items() if len(v) > 1}
    assert not dup, "kernels defined in several objects: %s" % list(dup.items())[:5]


def test_k16_scan_kernels_keep_registers():
    """The K = 16 scan kernels of the unforced configurations (at most two
    query tiles per wave on the 32-wide tiles) keep everything in registers:
    a small change to the flush code once made the compiler aim at one more
    wave per SIMD and spill the bf16 filter to scratch, three times slower.
    Reads the register summaries of the device assembly the build keeps."""
    asms = sorted(glob.glob(os.path.join(ROOT, "_build", "hn_scan_*", "*-gfx950.s")))
    asms = [a for a in asms if "multi" not in os.path.basename(a)]
    if not asms:
        pytest.skip("no device assembly (run the build first)")
    checked, spilled = 0, []
    for a in asms:
        name = None
        with open(a) as fh:
            for line in fh:
                m = re.match(r"^(_ZN2hn11scan_kernelI\S*Tile32ILi16EEELi([0-9]+)E\S*):\s", line)
                if m:
                    name = m.group(1) if int(m.group(2)) <= 2 else None
                    continue
                if name and line.startswith("; ScratchSize:"):
                    checked += 1
                    if int(line.split(":")[1]) > 0:
                        spilled.append(name)
                    name = None
    assert checked >= 8, "expected the K = 16 scan kernels in the assembly (found %d)" % checked
    assert not spilled, "scan kernels spilling to scratch: %s" % spilled
