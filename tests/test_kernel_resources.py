"""The compiler's resource report of the last build: no kernel of the hot
path may use per-lane scratch memory.  Scratch appears when the compiler
keeps captured variables or an argument structure in memory (for instance a
helper lambda left out of line), and it slows a kernel several times over."""
import os
import re

import pytest

from paper_2001_07089_amd import build as B


def _kernels():
    if not os.path.exists(B.RESOURCES):
        pytest.skip("no resource report (library not built in this tree)")
    out, cur = {}, None
    for line in open(B.RESOURCES):
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?:\s+(\d+)", line)
        if cur and m:
            out[cur][m.group(1).strip()] = int(m.group(2))
    return out


def test_no_hot_kernel_uses_scratch():
    ks = _kernels()
    hot = [k for k in ks if re.search(r"k_rb_|k_force_|k_kick|k_drift|k_rdf_|k_van_hove|k_msd_", k)]
    assert len(hot) >= 12
    bad = {k: ks[k].get("ScratchSize") for k in hot if ks[k].get("ScratchSize", 0) != 0}
    assert not bad, bad
