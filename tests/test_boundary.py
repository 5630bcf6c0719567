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


def test_header_has_north_star_entry_points():
    names = _declared()
    for n in ("md_init", "md_build_cells", "md_forces", "md_step_nve", "md_step_nvt", "md_rdf", "md_msd"):
        assert n in names


def _reps(ns, rho=1.2, T=1.0):
    return md.make_replicas([(n, W.n_a_for(n), W.box_for(n, rho), T, 7 + i) for i, n in enumerate(ns)])


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
        md.md_init(cfg, _reps([500]), st, 0)
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
