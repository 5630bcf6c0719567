"""md_init_static, the entry point for callers that cannot allocate device
memory, against md_init on the same input: its context works in a fixed
per-device array instead of a caller's or the library's workspace, and must
give what md_init's context gives, bit for bit (the same kernels on the same
layout).  Two calls in a row, the second with fewer particles in the array the
first one used; each is destroyed before the next."""
import math
import sys

import numpy as np
import pytest

from paper_2001_07089_amd import md
from paper_2001_07089_amd import workload as W

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(sizes, seed):
    reps, pos, vel = [], [[], [], []], [[], [], []]
    for k, n in enumerate(sizes):
        L = W.box_for(n, 1.2)
        reps.append((n, W.n_a_for(n), L, 0.8, seed + k))
        x, y, z = W.lattice_config(n, L, seed + k, 0.08)
        v = W.gaussian_velocities(n, math.sqrt(0.8), seed + 10 + k)
        for i, a in enumerate((x, y, z)):
            pos[i].append(a)
        for i, a in enumerate(v):
            vel[i].append(a)
    return reps, [np.concatenate(p) for p in pos], [np.concatenate(v) for v in vel]


def static_context(ref, pos, vel):
    """Caller arrays like md.System's, and a context from md_init_static."""
    torch = ref.torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t = {k: torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")
             for k, a in zip(KEYS[:6], list(pos) + list(vel))}
        for k in KEYS[6:]:
            t[k] = torch.zeros(ref.n_total, dtype=torch.float64, device="cuda")
        img = torch.zeros((3, ref.n_total), dtype=torch.int32, device="cuda")
    st = md.State()
    for k in KEYS:
        setattr(st, k, t[k].data_ptr())
    st.img = img.data_ptr()
    stream.synchronize()
    ctx = md.md_init_static(ref.cfg, ref.reps, st, stream.cuda_stream)
    return ctx, stream, t, img


def host(stream, t, img):
    stream.synchronize()
    return {k: t[k].cpu().numpy() for k in KEYS}, img.cpu().numpy()


@pytest.mark.parametrize("prec", ["mixed_fixed", "fp64"])
def test_static_context_equals_md_init_twice(prec):
    for call, sizes in enumerate(([3000, 1200], [800])):
        log(f"case md_init_static {prec} call {call}: N = {sizes}")
        reps, pos, vel = inputs(sizes, 40 + call)
        ref = md.System(reps, precision=prec, positions=pos, velocities=vel)
        ctx, stream, t, img = static_context(ref, pos, vel)
        a, _ = host(stream, t, img)
        b = ref.numpy()
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (call, k)
        md.md_step_nve(ctx, 60)
        ref.step_nve(60)
        a, ia = host(stream, t, img)
        b = ref.numpy()
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (call, k)
        assert np.array_equal(ia, ref.images())
        assert md.md_status(ctx) == 0
        # the array is in use: a second static context on this device is refused
        with pytest.raises(md.KamdError) as e:
            md.md_init_static(ref.cfg, ref.reps, ref.state, stream.cuda_stream)
        assert e.value.code == md.KAMD_ESTATE
        md.md_destroy(ctx)
        ref.close()


def test_static_context_refuses_a_system_beyond_the_array():
    n = 200000
    reps = md.make_replicas([(n, W.n_a_for(n), W.box_for(n, 1.2), 0.8, 1)])
    cfg = md.make_config("mixed_fixed", init_mode=md.INIT_LATTICE)
    assert md.md_workspace_size(cfg, reps) > 64 << 20
    with pytest.raises(md.KamdError) as e:
        md.md_init_static(cfg, reps, md.State(), 0)
    assert e.value.code == md.KAMD_ENOMEM
    assert b"static array" in md.lib().md_last_error(None)


def test_a_static_context_moved_to_a_caller_workspace_frees_the_array():
    """md_set_workspace moves a static context into the caller's block; the
    static array is then free for the next md_init_static, and the moved
    context still steps as md_init's does."""
    reps, pos, vel = inputs([1500], 77)
    ref = md.System(reps, precision="mixed_fixed", positions=pos, velocities=vel)
    ctx, stream, t, img = static_context(ref, pos, vel)
    torch = ref.torch
    need = md.md_workspace_needed(ctx)
    with torch.cuda.stream(stream):
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stream.synchronize()
    md.md_set_workspace(ctx, ws.data_ptr(), need)
    ctx2, stream2, t2, img2 = static_context(ref, pos, vel)  # the array is free again
    md.md_step_nve(ctx, 40)
    md.md_step_nve(ctx2, 40)
    ref.step_nve(40)
    b = ref.numpy()
    for c, s_, tt, ii in ((ctx, stream, t, img), (ctx2, stream2, t2, img2)):
        a, _ = host(s_, tt, ii)
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k
        assert md.md_status(c) == 0
    md.md_destroy(ctx2)
    md.md_destroy(ctx)
    ref.close()
