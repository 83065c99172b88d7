"""Every kernel of the built library is defined in exactly one translation
unit.  A kernel template instantiated in two units gets two device copies
behind one host launch stub, and which copy a launch runs is then up to the
runtime's registration order; with identical sources that is harmless, but it
hides any difference between the units' builds.  The check reads the symbol
tables of the objects the build leaves in _build/ (skipped before a build)."""
import glob
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
