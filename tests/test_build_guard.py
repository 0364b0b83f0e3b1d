"""The built kernels stay inside the resource envelope that has run cleanly
on MI355X: no kernel's private (scratch) segment above the build's limit."""
import glob
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1904_07400_amd", "_build")


def test_kernel_scratch_within_limit():
    objs = sorted(glob.glob(os.path.join(BUILD, "sg_kernels_p*.o")))
    if not objs:
        pytest.skip("kernel objects not built")
    from paper_1904_07400_amd import build as b
    res = [r for o in objs for r in b.kernel_resources(o)]
    names = [r[0] for r in res]
    # every per-step kernel of the forward and adjoint path is present
    for k in ("k_row_fwd", "k_col", "k_row_inv", "k_col_adj", "k_row_c2r", "k_weights", "k_spec_col"):
        assert any(k in n for n in names), k
    worst = max(res, key=lambda r: r[1])
    assert worst[1] <= b.SCRATCH_LIMIT, worst
    # no workgroup asks for more LDS than the 160 KiB of a CU
    assert max(r[2] for r in res) <= 160 * 1024
