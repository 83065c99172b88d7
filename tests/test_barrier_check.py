"""The build-time barrier check (paper_2606_27280_amd/csrc/check_barriers.py)
on small hand-written gfx950 assembly: a loop whose exit accumulates an exec
mask must not hold a work-group barrier, whichever way the compiler lays out
and annotates the loop's blocks."""
import importlib.util
import os

HERE = os.path.dirname(os.path.abspath(__file__))
spec = importlib.util.spec_from_file_location(
    "check_barriers",
    os.path.join(HERE, "..", "paper_2606_27280_amd", "csrc", "check_barriers.py"))
cb = importlib.util.module_from_spec(spec)
# the module runs its command-line part only under __main__
spec.loader.exec_module(cb)


def _kernel(body):
    return ["_Z6kernelv:", *body, ".Lfunc_end0:"]


# Exit block laid out before the header; the header's loop annotation sits on
# the comment line after its label (the label carries a long block name).
DIVERGENT_EXIT_BEFORE_HEADER = _kernel([
    "\ts_branch .LBB0_2",
    ".LBB0_1:                               ; %Flow12",
    "\ts_or_b64 exec, exec, s[6:7]",
    "\ts_andn2_b64 exec, exec, s[74:75]",
    "\ts_cbranch_execz .LBB0_9",
    ".LBB0_2:                               ; %some.long.block.name.exit",
    "                                        ; =>This Loop Header: Depth=1",
    "\ts_and_saveexec_b64 s[6:7], s[14:15]",
    ".LBB0_3:                               ;   in Loop: Header=BB0_2 Depth=1",
    "\ts_waitcnt lgkmcnt(0)",
    "\ts_barrier",
    "\ts_branch .LBB0_1",
    ".LBB0_9:",
    "\ts_endpgm",
])

# Divergent inner loop whose header annotation lists its parent after the label.
DIVERGENT_INNER = _kernel([
    ".LBB1_1:                               ; =>This Loop Header: Depth=1",
    "\ts_nop 0",
    ".LBB1_2:                               ; %inner",
    "                                        ;   Parent Loop BB1_1 Depth=1",
    "                                        ; =>  This Inner Loop Header: Depth=2",
    "\ts_barrier",
    "\ts_andn2_b64 exec, exec, s[8:9]",
    "\ts_cbranch_execnz .LBB1_2",
    ".LBB1_3:                               ;   in Loop: Header=BB1_1 Depth=1",
    "\ts_cbranch_scc1 .LBB1_1",
    "\ts_endpgm",
])

# Uniform loop (scalar exit) with a barrier, and a divergent loop without one.
CLEAN = _kernel([
    ".LBB2_1:                               ; =>This Loop Header: Depth=1",
    "\ts_barrier",
    "\ts_cmp_ge_i32 s88, s57",
    "\ts_cbranch_scc1 .LBB2_1",
    ".LBB2_2:                               ; =>This Loop Header: Depth=1",
    "\tv_add_u32_e32 v1, 1, v1",
    "\ts_andn2_b64 exec, exec, s[8:9]",
    "\ts_cbranch_execnz .LBB2_2",
    "\ts_endpgm",
])


def test_flags_exit_laid_out_before_header():
    n, flagged = cb.check(DIVERGENT_EXIT_BEFORE_HEADER)
    assert n == 1 and [h for _, h in flagged] == ["BB0_2"]


def test_flags_divergent_inner_loop_and_its_parent_barrier():
    _, flagged = cb.check(DIVERGENT_INNER)
    assert [h for _, h in flagged] == ["BB1_2"]


def test_uniform_loop_with_barrier_passes():
    n, flagged = cb.check(CLEAN)
    assert n == 1 and flagged == []


def test_device_globals_are_not_kernels():
    """A device global's label (no function end) is skipped, not parsed as a
    kernel."""
    asm = DIVERGENT_INNER + ["\t.type\t_ZN2hn7scratchE,@object", "_ZN2hn7scratchE:",
                             "\t.zero\t64"]
    total, flagged = cb.check(asm)
    assert len(flagged) >= 1
