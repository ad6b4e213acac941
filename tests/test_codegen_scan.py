"""The device code holds no spill ahead of an exec-mask restore inside a loop.

hipcc for gfx950 can put the spill of a value leaving a divergent region in
the region's join block before the exec restore, so the lanes that skipped
the region reload a stale value (wrong adjoint cotangents in one variant
before the adjoint stopped carrying the node time across the reverse pass).
The scanner is checked on hand-written assembly first, then run over the
library's own device assembly (compiled here, no GPU needed)."""
import os
import tempfile

from paper_2609_28458_amd import codegen_scan as cs

# A kernel whose loop holds a divergent region: the join block .LBB0_3 is
# reached by s_cbranch_execz and spills v[8:9] before restoring exec.
_BAD = """\
_Z6kernelv:                             ; @_Z6kernelv
.LBB0_1:                                ; =>This Loop Header: Depth=1
\tv_cmp_gt_f64_e64 s[0:1], v[8:9], v[2:3]
\ts_and_saveexec_b64 s[10:11], s[0:1]
\ts_cbranch_execz .LBB0_3
; %bb.2:                                ;   in Loop: Header=BB0_1 Depth=1
\tv_mov_b32_e32 v9, 0xfff00000
.LBB0_3:                                ;   in Loop: Header=BB0_1 Depth=1
\tscratch_store_dwordx2 off, v[8:9], off offset:16 ; 8-byte Folded Spill
\ts_or_b64 exec, exec, s[10:11]
\ts_cbranch_scc1 .LBB0_1
\ts_endpgm
"""


def test_scanner_flags_a_spill_ahead_of_the_exec_restore():
    hits = cs.scan_text(_BAD)
    assert len(hits) == 1
    assert hits[0].block == ".LBB0_3" and hits[0].in_loop
    assert hits[0].spills[0].startswith("scratch_store_dwordx2")


def test_scanner_passes_the_same_spill_after_the_restore():
    ok = _BAD.replace(
        "\tscratch_store_dwordx2 off, v[8:9], off offset:16 ; 8-byte Folded Spill\n"
        "\ts_or_b64 exec, exec, s[10:11]\n",
        "\ts_or_b64 exec, exec, s[10:11]\n"
        "\tscratch_store_dwordx2 off, v[8:9], off offset:16 ; 8-byte Folded Spill\n")
    assert cs.scan_text(ok) == []


def test_scanner_ignores_lane_writes_and_region_bodies():
    # v_writelane ignores exec; a block that is not an execz target is the
    # region's own body, whose stores belong under the narrowed mask.
    lane = _BAD.replace("scratch_store_dwordx2 off, v[8:9], off offset:16 ; 8-byte Folded Spill",
                        "v_writelane_b32 v255, s2, 15")
    assert cs.scan_text(lane) == []
    body = _BAD.replace("s_cbranch_execz .LBB0_3", "s_cbranch_execz .LBB0_4")
    assert cs.scan_text(body) == []


def test_scanner_marks_joins_outside_loops():
    flat = _BAD.replace(";   in Loop: Header=BB0_1 Depth=1", "")
    hits = cs.scan_text(flat)
    assert len(hits) == 1 and not hits[0].in_loop


def test_library_device_code_has_no_spill_ahead_of_an_exec_restore_in_a_loop():
    with tempfile.TemporaryDirectory() as d:
        paths = cs.device_asm(d)
        assert all(os.path.getsize(p) > 0 for p in paths)
        hits = [h for p in paths for h in cs.scan(p)]
    inside = [(h.kernel, h.block, h.spills) for h in hits if h.in_loop]
    assert inside == []
    # Outside loops only the static-schedule start of the persistent forward
    # kernels, whose masked-off lanes never become live.
    for h in hits:
        assert "solve_kernel" in h.kernel or "sens_kernel" in h.kernel, h.kernel
