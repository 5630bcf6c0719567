"""C-ABI boundary checks that need no GPU: the library loads, exports every
function declared in include/kamd.h, and its host-side validation, footprint
and admission logic behave as documented."""
import os
import re

import numpy as np

import pytest

from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "kamd.h")).read()
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = md.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(md.EXPORTED)


def test_header_declares_the_hot_path_entry_points():
    names = _declared()
    for n in ("md_init", "md_build_cells", "md_forces", "md_step_nve", "md_step_nvt", "md_rdf", "md_msd"):
        assert n in names


def _reps(ns, rho=1.2, T=1.0):
    return md.make_replicas([(n, W.n_a_for(n), W.box_for(n, rho), T, 7 + i) for i, n in enumerate(ns)])


def test_workspace_holds_packed_positions_for_fp64_only():
    """FP64 contexts keep two packed (x, y, z, 0) position buffers of 32 B per
    padded slot for the fused steps; the mixed precisions gather the u32
    mirror and keep none.  Every type segment is padded to 64 slots."""
    ns = [1000, 333, 4097]
    npad = 0
    for n in ns:
        na = W.n_a_for(n)
        npad += -(-na // 64) * 64 + -(-(n - na) // 64) * 64
    f = md.md_workspace_size(md.make_config("fp64"), _reps(ns))
    for prec in ("mixed", "mixed_fixed"):
        m = md.md_workspace_size(md.make_config(prec), _reps(ns))
        assert f - m == 64 * npad, prec


def test_workspace_size_scales_with_particles():
    cfg = md.make_config()
    a = md.md_workspace_size(cfg, _reps([1000]))
    b = md.md_workspace_size(cfg, _reps([8000]))
    assert 0 < a < b
    # list rows dominate: a few hundred bytes to ~1.5 kB per particle
    assert 200 * 8000 < b < 3000 * 8000


def test_validation_errors():
    cfg = md.make_config()
    with pytest.raises(md.KamdError) as e:
        md.md_workspace_size(cfg, md.make_replicas([(100, 80, 4.0, 1.0, 1)]))  # L/2 < r_c
    assert e.value.code == md.KAMD_EBOX
    with pytest.raises(md.KamdError) as e:
        md.md_workspace_size(cfg, md.make_replicas([(100, 120, 9.0, 1.0, 1)]))
    assert e.value.code == md.KAMD_EINVAL
    bad = md.make_config(dt=0.0)
    with pytest.raises(md.KamdError) as e:
        md.md_workspace_size(bad, _reps([500]))
    assert e.value.code == md.KAMD_EINVAL
    bad = md.make_config(precision=7)
    with pytest.raises(md.KamdError):
        md.md_workspace_size(bad, _reps([500]))


def test_planar_cell_grid_is_one_layer():
    """A planar system bins into nc^2 cells: at 2^20 particles (L = 933) the
    workspace (about 1.1 kB per particle: state, list, MSD origins, RDF and
    staging) hardly depends on the cell division, where a cubic grid would
    need 2 * 333^3 cells at division 1 and 2 * 666^3 at division 2, i.e. 3.8
    and 30 GB of cell tables."""
    wl = W.ka_planar(1 << 20, 0.4)
    r = wl.replicas[0]
    reps = md.make_replicas([(r.n, r.n_a, r.box, r.temperature, r.seed)])
    one = md.md_workspace_size(md.make_config(precision="mixed_fixed", dim=2, cell_div=1), reps)
    two = md.md_workspace_size(md.make_config(precision="mixed_fixed", dim=2, cell_div=2), reps)
    assert one < 3 << 29 and two < 3 << 29
    # division 1: 2 * 333^2 cells; division 2: 2 * 666^2; 52 bytes per cell
    # (count, start and end for each of 4 sub-cells, and the segment index)
    assert abs(two - one) < 52 * 2 * 700 ** 2


def test_cell_grid_limits():
    """Cells per edge are capped (wider cells stay correct), and a plan whose
    cell grid would exceed 2^26 cells in all is refused, not truncated."""
    cfg = md.make_config()
    sparse = [(1000, 800, 800.0, 1.0, 3 + i) for i in range(3)]  # 2 * 256^3 = 2^25 cells each after the cap
    two = md.md_workspace_size(cfg, md.make_replicas(sparse[:2]))
    assert two < 53 * (1 << 26)  # 52 bytes per cell, and the rest of the plan
    with pytest.raises(md.KamdError) as e:
        md.md_workspace_size(cfg, md.make_replicas(sparse))
    assert e.value.code == md.KAMD_EINVAL and "cell grid" in str(e.value)
    adm, cnt = md.md_admit(cfg, md.make_replicas(sparse), 10 ** 12)
    assert cnt == 2 and adm.tolist() == [1, 1, 0]


def test_admission_by_footprint():
    cfg = md.make_config()
    reps = _reps([2000, 4000, 8000, 3000])
    one = md.md_workspace_size(cfg, _reps([2000]))
    adm, cnt = md.md_admit(cfg, reps, 10 ** 12)
    assert cnt == 4 and adm.tolist() == [1, 1, 1, 1]
    adm, cnt = md.md_admit(cfg, reps, 1)
    assert cnt == 0
    adm, cnt = md.md_admit(cfg, reps, int(one * 1.05))
    assert adm[0] == 1 and cnt >= 1
    assert adm.sum() == cnt


def test_init_without_device_reports_hip_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    cfg = md.make_config()
    st = md.State()
    with pytest.raises(md.KamdError) as e:
        md.md_init(cfg, _reps([500]), st, 0, 0, 0)
    assert e.value.code in (md.KAMD_EINVAL, md.KAMD_EHIP)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(md, "_lib", None)
    monkeypatch.setattr(md, "LIB_PATH", "/nonexistent/libkamd.so")
    with pytest.raises(RuntimeError):
        md.lib()


def test_log_schedule_matches_oracle_and_definition():
    """Host-side log schedule of the library against the oracle's loop (Sec.
    VI.B.1) and against its definition: distinct, increasing, inside [1, n_md],
    first step round(t0), last step n_md."""
    import oracle as O
    for n_md, t0, kmax in [(1000, 1.0, 60), (10000, 1.0, 60), (100000, 1.0, 60), (500, 2.5, 30),
                           (7, 1.0, 10), (20000, 10.0, 40)]:
        got = md.md_log_schedule(n_md, t0, kmax)
        ref = O.log_schedule(n_md, t0, kmax)
        assert np.array_equal(got, ref), (n_md, t0, kmax)
        assert np.all(np.diff(got) > 0) and got[0] == round(t0) and got[-1] == n_md
    assert len(md.md_log_schedule(1000, 1.0, 60)) == 50
    # degenerate growth factor A = 1 (n_md == t0): the single step t0
    assert list(md.md_log_schedule(1, 1.0, 5)) == [1]
    with pytest.raises(md.KamdError):
        md.md_log_schedule(0, 1.0, 60)
    with pytest.raises(md.KamdError):
        md.md_log_schedule(100, 0.2, 60)
