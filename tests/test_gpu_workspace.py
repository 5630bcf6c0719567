"""The boundary's memory contract and the neighbour-list self-heal.

A context works in one device workspace, md_workspace_size bytes, that the
caller may own (here a torch tensor); the library never frees a caller's
workspace.  A list that outgrows its rows (the LAMMPS-style rebuild check of
Sec. IV.B keeps the pair set exact only while every list fits) is healed by
the eager calls: the list grows and the call is redone, so forces and
trajectories equal those of a context whose lists never overflowed.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def liquid(n, T=1.0, seed=21):
    L = W.box_for(n, 1.2)
    na = W.n_a_for(n)
    x, y, z = W.lattice_config(n, L, seed, 0.08)
    vx, vy, vz = W.gaussian_velocities(n, math.sqrt(T), seed + 1)
    st = O.State(x, y, z, vx, vy, vz, na, L)
    st.compute_forces()
    O.run(st, 0.001, 150, nb=5, T=T, seed=seed)
    return st


def make(st, prec, **kw):
    return md.System([(st.n, st.na, st.L, 1.0, 3)], precision=prec, positions=(st.x, st.y, st.z),
                     velocities=(st.vx, st.vy, st.vz), **kw)


def normwise(a, b):
    return math.sqrt(sum(np.sum((a[k] - b[k]) ** 2) for k in range(3)) / sum(np.sum(b[k] ** 2) for k in range(3)))


def test_caller_workspace_is_exactly_the_reported_size():
    st = liquid(2000)
    s = make(st, "mixed_fixed")
    assert s.ws_bytes == md.md_workspace_size(s.cfg, s.reps)
    assert s.ws.numel() == s.ws_bytes
    assert md.md_workspace_needed(s.ctx) == s.ws_bytes
    s.close()
    # one byte short is refused; a library-owned workspace needs no argument
    torch = s.torch
    need = md.md_workspace_size(s.cfg, s.reps)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(md.KamdError) as e:
        md.md_init(s.cfg, s.reps, s.state, s.stream.cuda_stream, small.data_ptr(), need - 256)
    assert e.value.code == md.KAMD_ENOMEM
    ctx = md.md_init(s.cfg, s.reps, s.state, s.stream.cuda_stream, 0, 0)
    assert md.md_workspace_needed(ctx) >= need
    md.md_destroy(ctx)


def test_larger_skin_grows_a_caller_workspace():
    st = liquid(3000)
    s = make(st, "fp64", skin=0.2)
    before = s.ws_bytes
    with pytest.raises(md.KamdError) as e:          # the raw call is refused ...
        md.md_set_list_params(s.ctx, 0.5, 2)
    assert e.value.code == md.KAMD_ENOMEM
    assert md.md_workspace_needed(s.ctx) > before
    s.set_list_params(0.5, 2)                         # ... the wrapper grows and repeats it
    assert s.ws_bytes > before
    s.forces()
    a = s.numpy()
    fx, fy, fz, _, _ = O.forces(st.x, st.y, st.z, st.na, st.L, "brute")
    assert normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz)) <= 1e-12
    assert md.md_stats(s.ctx)["skin"] == 0.5
    s.close()


@pytest.mark.parametrize("owned", [False, True])
def test_list_overflow_heals(owned):
    """list_capacity 0.05: the first build overflows.  The lists grow, forces
    equal the oracle's, and 200 eager MIXED_FIXED steps equal (bitwise) those
    of a context built with the default capacity."""
    st = liquid(4000)
    ref = make(st, "mixed_fixed")
    # owned: the library's own workspace, reallocated as the list grows;
    # else the caller's, with room for the list at the default capacity
    s = make(st, "mixed_fixed", list_capacity=0.05, own_workspace=not owned)
    assert md.md_status(s.ctx) == 0              # healed: no overflow bit left
    rows = md.md_stats(s.ctx)["list_rows"]
    log(f"  healed list rows {rows}")
    a = s.numpy()
    fx, fy, fz, _, _ = O.forces(st.x, st.y, st.z, st.na, st.L, "brute")
    assert normwise((a["ax"], a["ay"], a["az"]), (fx, fy, fz)) <= 1e-5
    b = ref.numpy()
    assert all(np.array_equal(a[k], b[k]) for k in ("ax", "ay", "az"))
    s.step_nve(200)
    ref.step_nve(200)
    a, b = s.numpy(), ref.numpy()
    assert all(np.array_equal(a[k], b[k]) for k in a)
    assert s.status() == 0
    s.close()
    ref.close()


def test_rdf_keeps_a_captured_graph():
    """The RDF grid lives in the workspace, so measuring at a new range no
    longer reallocates and drops the captured step graph."""
    st = liquid(3000)
    s = make(st, "mixed_fixed")
    s.capture(50)
    h1 = s._host(s.rdf(0.05, 40))
    h2 = s._host(s.rdf(0.02, 300))   # a wider range: another grid
    s.launch()
    s.launch()
    assert s.status() == 0
    a = s.numpy()
    sl = slice(0, st.n)
    ref = O.rdf_hist(st.x, st.y, st.z, st.na, st.L, 0.05, 40)
    assert np.array_equal(h1[0].astype(np.uint64), ref)
    ref2 = O.rdf_hist(st.x, st.y, st.z, st.na, st.L, 0.02, 300)
    assert np.array_equal(h2[0].astype(np.uint64), ref2)
    assert md.md_stats(s.ctx)["steps"] == 100
    s.close()
