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


# The opt-in window variant of the mixed step kernel (template argument STAGE
# = true, ENERGY = false) is held to the register count that its LDS use
# allows (five wavefronts per SIMD); the compiler then keeps two 8-byte values
# in scratch (20 bytes per lane), stored once per wavefront, outside the pair
# loops.  The variant runs faster so than without the bound; it may use at
# most this much.
STAGED_STEP = re.compile(r"k_force_mixedILb[01]ELb0ELb[01]ELb1E")
STAGED_SCRATCH_MAX = 32


def test_no_hot_kernel_uses_scratch():
    ks = _kernels()
    hot = [k for k in ks if re.search(r"k_rb_|k_force_|k_kick|k_drift|k_rdf_|k_van_hove|k_msd_", k)]
    assert len(hot) >= 12
    bad = {k: ks[k].get("ScratchSize") for k in hot
           if ks[k].get("ScratchSize", 0) != 0 and not STAGED_STEP.search(k)}
    assert not bad, bad
    staged = [k for k in hot if STAGED_STEP.search(k)]
    assert staged
    over = {k: ks[k].get("ScratchSize") for k in staged if ks[k].get("ScratchSize", 0) > STAGED_SCRATCH_MAX}
    assert not over, over
