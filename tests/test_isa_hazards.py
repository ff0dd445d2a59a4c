"""Wait states between matrix-core products and their readers in the built
kernels (no GPU: the kernels are compiled to gfx950 assembly and every path
is walked)."""
import os
import shutil

import pytest

from paper_2108_07001_amd import isa_scan
from paper_2108_07001_amd.build import HIPCC

LISTING = """\
_Zkernel:
\tv_mfma_f32_32x32x16_f16 v[12:27], v[0:3], v[4:7], v[12:27]
\ts_cbranch_scc1 .LBB0_2
; %bb.1:
\tglobal_load_dwordx4 v[0:3], v[40:41], off
\tv_mov_b32_e32 v30, 0
\tv_mov_b32_e32 v31, 0
\tv_mov_b32_e32 v32, 0
\tv_mov_b32_e32 v33, 0
\tv_mov_b32_e32 v34, 0
\tv_mov_b32_e32 v35, 0
\tv_mov_b32_e32 v36, 0
\tv_mov_b32_e32 v37, 0
\tv_mov_b32_e32 v38, 0
\tv_mov_b32_e32 v39, 0
.LBB0_2:
\t{pad}
\tv_exp_f32_e32 v50, v12
\ts_endpgm
.Lfunc_end0:
"""


def test_scanner_flags_a_short_branch_path():
    # the fall-through path has 12 wait states, the taken branch only 1
    bad = isa_scan.short_paths(LISTING.format(pad="s_nop 0"))
    assert len(bad) == 1 and "2 wait states" in bad[0] and "v_exp_f32" in bad[0]


def test_scanner_accepts_padded_paths():
    assert isa_scan.short_paths(LISTING.format(pad="s_nop 10")) == []


def test_scanner_leaves_paths_through_another_product():
    listing = LISTING.format(pad="v_mfma_f32_32x32x16_f16 v[60:75], v[0:3], v[4:7], v[60:75]")
    assert isa_scan.short_paths(listing) == []


def test_scanner_sees_register_ranges_and_writes():
    listing = LISTING.replace("v_exp_f32_e32 v50, v12", "v_mov_b32_e32 v27, 0").format(pad="s_nop 0")
    assert len(isa_scan.short_paths(listing)) == 1
    listing = LISTING.replace("v_exp_f32_e32 v50, v12", "v_mov_b32_e32 v28, 0").format(pad="s_nop 0")
    assert isa_scan.short_paths(listing) == []


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not available")
def test_library_kernels_have_no_short_paths():
    bad = isa_scan.check()
    assert not bad, "\n".join(bad[:20])
