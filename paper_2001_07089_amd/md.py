"""Thin ctypes binding of the C ABI in ``include/kamd.h``.

Each ``md_*`` function here marshals its arguments and calls the function of
the same name in ``_lib/libkamd.so``; all computation happens in the HIP
kernels behind it.  A non-zero return code raises :class:`KamdError` with the
library's message.  PyTorch is used only to own device memory and to provide
the HIP stream (``System`` below).

There is no fallback: if the library is missing or cannot be loaded, every
call raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libkamd.so")

KAMD_OK, KAMD_EINVAL, KAMD_ENOMEM, KAMD_EHIP, KAMD_EDEVICE, KAMD_EBOX, KAMD_ESTATE = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_MIXED, PREC_MIXED_FIXED = 0, 1, 2
F_FORCE, F_ENERGY, F_VIRIAL = 1, 2, 4
NVT_STOCHASTIC, NVT_NOSE_HOOVER = 0, 1
INIT_GIVEN, INIT_RSA, INIT_LATTICE = 0, 1, 2
DEV_NONFINITE, DEV_LIST_OVERFLOW, DEV_FORCE_RANGE, DEV_LIST_FORMAT, DEV_RUNAWAY = 1, 2, 4, 8, 16
PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED, "mixed_fixed": PREC_MIXED_FIXED}

# Kob-Andersen parameters (Sec. II.B), pair order AA, AB, BB.
KA_EPS = (1.0, 1.5, 0.5)
KA_SIGMA = (1.0, 0.8, 0.88)
KA_RC_FACTOR = 2.5

EXPORTED = ("md_workspace_size", "md_admit", "md_init", "md_build_cells", "md_forces", "md_step_nve",
            "md_step_nvt", "md_rdf", "md_msd", "md_observables", "md_thermostat_state", "md_sync",
            "md_import", "md_graph_capture", "md_graph_launch", "md_autotune", "md_set_list_params",
            "md_stats", "md_get_state", "md_set_state", "md_profile", "md_status", "md_last_error", "md_destroy",
            "md_log_schedule", "md_set_temperature", "md_scale_velocities", "md_van_hove",
            "md_observables_now", "md_clear_samples", "md_workspace_needed", "md_set_workspace",
            "md_init_static", "md_set_force_kernel", "md_clear_status")


class KamdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kamd error {code}: {msg}")
        self.code = code


class Model(C.Structure):
    _fields_ = [("eps", C.c_double * 3), ("sigma", C.c_double * 3), ("rc_factor", C.c_double)]


class Replica(C.Structure):
    _fields_ = [("offset", C.c_int64), ("n", C.c_int32), ("n_a", C.c_int32), ("box", C.c_double),
                ("temperature", C.c_double), ("seed", C.c_uint64)]


class State(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "img")]


class Config(C.Structure):
    _fields_ = [("model", Model), ("precision", C.c_int32), ("dt", C.c_double), ("skin", C.c_double),
                ("init_mode", C.c_int32), ("min_dist", C.c_double), ("cell_div", C.c_int32),
                ("list_capacity", C.c_double), ("auto_sync", C.c_int32), ("dim", C.c_int32),
                ("pe_unshifted", C.c_int32), ("sample_every", C.c_int32), ("sample_capacity", C.c_int32),
                ("msd_slots", C.c_int32)]


_lib = None


def lib():
    """Load ``_lib/libkamd.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32, f64, u32 = C.c_int32, C.c_double, C.c_uint32
        sig = {
            "md_workspace_size": [C.POINTER(Config), P, i32, C.POINTER(C.c_size_t)],
            "md_admit": [C.POINTER(Config), P, i32, C.c_size_t, P, C.POINTER(i32)],
            "md_init": [C.POINTER(P), C.POINTER(Config), P, i32, C.POINTER(State), P, C.c_size_t, P],
            "md_workspace_needed": [P, C.POINTER(C.c_size_t)],
            "md_init_static": [C.POINTER(P), C.POINTER(Config), P, i32, C.POINTER(State), P],
            "md_set_workspace": [P, P, C.c_size_t],
            "md_build_cells": [P],
            "md_forces": [P, u32, P],
            "md_step_nve": [P, i32],
            "md_step_nvt": [P, i32, i32, i32, f64],
            "md_rdf": [P, f64, i32, P],
            "md_msd": [P, i32, i32, P],
            "md_observables": [P, P, i32, C.POINTER(i32)],
            "md_observables_now": [P, P],
            "md_clear_samples": [P],
            "md_thermostat_state": [P, P],
            "md_sync": [P],
            "md_import": [P],
            "md_graph_capture": [P, i32, i32, i32, i32, f64],
            "md_graph_launch": [P],
            "md_autotune": [P, i32, P],
            "md_set_list_params": [P, f64, i32],
            "md_set_force_kernel": [P, i32, i32],
            "md_clear_status": [P],
            "md_stats": [P, P],
            "md_get_state": [P, P, C.POINTER(C.c_size_t)],
            "md_set_state": [P, P, C.c_size_t],
            "md_status": [P, C.POINTER(u32)],
            "md_profile": [P, i32, P],
            "md_destroy": [P],
            "md_log_schedule": [i32, f64, i32, P, i32, C.POINTER(i32)],
            "md_set_temperature": [P, P],
            "md_van_hove": [P, i32, f64, i32, P],
            "md_scale_velocities": [P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.md_last_error.argtypes = [P]
        L.md_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(code, ctx=None):
    if code != KAMD_OK:
        msg = lib().md_last_error(ctx)
        raise KamdError(code, msg.decode() if msg else "")
    return code


def make_model(eps=KA_EPS, sigma=KA_SIGMA, rc_factor=KA_RC_FACTOR) -> Model:
    m = Model()
    for p in range(3):
        m.eps[p] = float(eps[p])
        m.sigma[p] = float(sigma[p])
    m.rc_factor = float(rc_factor)
    return m


def make_config(precision="fp64", dt=0.005, skin=0.3, init_mode=INIT_GIVEN, min_dist=0.8, cell_div=1,
                list_capacity=0.0, auto_sync=1, model=None, dim=3, pe_unshifted=False, sample_every=0,
                sample_capacity=0, msd_slots=0) -> Config:
    c = Config()
    c.model = model if model is not None else make_model()
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.dt = float(dt)
    c.skin = float(skin)
    c.init_mode = int(init_mode)
    c.min_dist = float(min_dist)
    c.cell_div = int(cell_div)
    c.list_capacity = float(list_capacity)
    c.auto_sync = int(auto_sync)
    c.dim = int(dim)
    c.pe_unshifted = 1 if pe_unshifted else 0
    c.sample_every = int(sample_every)
    c.sample_capacity = int(sample_capacity)
    c.msd_slots = int(msd_slots)
    return c


def make_replicas(reps):
    """reps: iterable of (n, n_a, box, temperature, seed) or objects with those attributes."""
    reps = list(reps)
    arr = (Replica * len(reps))()
    off = 0
    for i, r in enumerate(reps):
        if isinstance(r, tuple):
            n, na, box, T, seed = r
        else:
            n, na, box, T, seed = r.n, r.n_a, r.box, r.temperature, r.seed
        arr[i].offset = off
        arr[i].n = int(n)
        arr[i].n_a = int(na)
        arr[i].box = float(box)
        arr[i].temperature = float(T)
        arr[i].seed = int(seed)
        off += int(n)
    return arr


# ------------------------------------------------------------- raw C calls
def md_workspace_size(cfg: Config, reps) -> int:
    b = C.c_size_t()
    _check(lib().md_workspace_size(C.byref(cfg), C.cast(reps, C.c_void_p), len(reps), C.byref(b)))
    return b.value


def md_admit(cfg: Config, reps, budget_bytes: int):
    adm = np.zeros(len(reps), np.int32)
    cnt = C.c_int32()
    _check(lib().md_admit(C.byref(cfg), C.cast(reps, C.c_void_p), len(reps), int(budget_bytes),
                          adm.ctypes.data, C.byref(cnt)))
    return adm, cnt.value


def md_init(cfg: Config, reps, state: State, stream: int, workspace: int = 0, ws_bytes: int = 0):
    """workspace: device address of ws_bytes caller-owned bytes, or 0 for a
    library-allocated workspace."""
    ctx = C.c_void_p()
    _check(lib().md_init(C.byref(ctx), C.byref(cfg), C.cast(reps, C.c_void_p), len(reps), C.byref(state),
                         C.c_void_p(workspace or None), int(ws_bytes), C.c_void_p(stream)))
    return ctx


def md_init_static(cfg: Config, reps, state: State, stream: int):
    """md_init in the library's fixed per-device array (no device allocation)."""
    ctx = C.c_void_p()
    _check(lib().md_init_static(C.byref(ctx), C.byref(cfg), C.cast(reps, C.c_void_p), len(reps), C.byref(state),
                                C.c_void_p(stream)))
    return ctx


def md_workspace_needed(ctx) -> int:
    b = C.c_size_t()
    _check(lib().md_workspace_needed(ctx, C.byref(b)), ctx)
    return b.value


def md_set_workspace(ctx, workspace: int, ws_bytes: int):
    _check(lib().md_set_workspace(ctx, C.c_void_p(workspace), int(ws_bytes)), ctx)


def md_build_cells(ctx):
    _check(lib().md_build_cells(ctx), ctx)


def md_forces(ctx, flags: int = F_FORCE, obs_ptr: int = 0):
    _check(lib().md_forces(ctx, int(flags), C.c_void_p(obs_ptr or None)), ctx)


def md_step_nve(ctx, nsteps: int):
    _check(lib().md_step_nve(ctx, int(nsteps)), ctx)


def md_step_nvt(ctx, nsteps: int, mode: int = NVT_STOCHASTIC, n_reassign: int = 50, tau: float = 0.5):
    _check(lib().md_step_nvt(ctx, int(nsteps), int(mode), int(n_reassign), float(tau)), ctx)


def md_rdf(ctx, dr: float, n_bins: int, hist_ptr: int):
    _check(lib().md_rdf(ctx, float(dr), int(n_bins), C.c_void_p(hist_ptr)), ctx)


def md_msd(ctx, op: int, slot: int, out_ptr: int = 0):
    _check(lib().md_msd(ctx, int(op), int(slot), C.c_void_p(out_ptr or None)), ctx)


def md_observables(ctx, n_rep: int, max_rows: int):
    """Sampled rows per replica: float64 [n_rep][rows][6] of {step, KE, PE, E_tot, T, W}."""
    out = np.zeros((n_rep, max(int(max_rows), 1), 6))
    rows = C.c_int32(0)
    _check(lib().md_observables(ctx, out.ctypes.data, int(max_rows), C.byref(rows)), ctx)
    return out[:, :rows.value].copy()


def md_clear_samples(ctx):
    _check(lib().md_clear_samples(ctx), ctx)


def md_observables_now(ctx, n_rep: int):
    out = np.zeros((n_rep, 6))
    _check(lib().md_observables_now(ctx, out.ctypes.data), ctx)
    return out


def md_thermostat_state(ctx, n_rep: int):
    out = np.zeros((n_rep, 2))
    _check(lib().md_thermostat_state(ctx, out.ctypes.data), ctx)
    return out


def md_sync(ctx):
    _check(lib().md_sync(ctx), ctx)


def md_import(ctx):
    _check(lib().md_import(ctx), ctx)


def md_graph_capture(ctx, nsteps, ensemble=0, mode=NVT_STOCHASTIC, n_reassign=50, tau=0.5):
    _check(lib().md_graph_capture(ctx, int(nsteps), int(ensemble), int(mode), int(n_reassign), float(tau)), ctx)


def md_graph_launch(ctx):
    _check(lib().md_graph_launch(ctx), ctx)


def md_autotune(ctx, probe_steps: int = 100):
    out = np.zeros(5)
    _check(lib().md_autotune(ctx, int(probe_steps), out.ctypes.data), ctx)
    return {"skin": float(out[0]), "cell_div": int(out[1]), "ms_per_step": float(out[2]),
            "windows": int(out[3]), "wg_size": int(out[4])}


def md_van_hove(ctx, slot: int, dr: float, n_bins: int, hist_ptr: int):
    _check(lib().md_van_hove(ctx, int(slot), float(dr), int(n_bins), hist_ptr), ctx)


def md_set_temperature(ctx, temperatures):
    t = np.ascontiguousarray(temperatures, np.float64)
    _check(lib().md_set_temperature(ctx, t.ctypes.data), ctx)


def md_scale_velocities(ctx, factors):
    f = np.ascontiguousarray(factors, np.float64)
    _check(lib().md_scale_velocities(ctx, f.ctypes.data), ctx)


def md_log_schedule(n_md: int, t0: float = 1.0, kmax: int = 60):
    """Log-spaced measurement steps (host only): numpy int32 array."""
    cnt = C.c_int32(0)
    _check(lib().md_log_schedule(int(n_md), float(t0), int(kmax), None, 0, C.byref(cnt)))
    out = np.zeros(max(cnt.value, 1), np.int32)
    _check(lib().md_log_schedule(int(n_md), float(t0), int(kmax), out.ctypes.data, int(cnt.value), C.byref(cnt)))
    return out[:cnt.value]


def md_set_list_params(ctx, skin: float, cell_div: int):
    _check(lib().md_set_list_params(ctx, float(skin), int(cell_div)), ctx)


def md_set_force_kernel(ctx, windows: int, wg_size: int = 0):
    _check(lib().md_set_force_kernel(ctx, int(windows), int(wg_size)), ctx)


def md_stats(ctx):
    out = np.zeros(14)
    _check(lib().md_stats(ctx, out.ctypes.data), ctx)
    keys = ("steps", "rebuilds", "n_total", "list_rows", "mean_list_len", "max_list_len", "skin", "cell_div",
            "mean_list_bytes", "windows", "staged_fraction", "wg_size", "mean_walked", "skin_min")
    return dict(zip(keys, out.tolist()))


def md_get_state(ctx) -> bytes:
    n = C.c_size_t()
    _check(lib().md_get_state(ctx, None, C.byref(n)), ctx)
    buf = C.create_string_buffer(n.value)
    _check(lib().md_get_state(ctx, buf, C.byref(n)), ctx)
    return buf.raw


def md_set_state(ctx, blob: bytes):
    _check(lib().md_set_state(ctx, blob, len(blob)), ctx)


def md_profile(ctx, nsteps: int):
    out = np.zeros(8)
    _check(lib().md_profile(ctx, int(nsteps), out.ctypes.data), ctx)
    keys = ("force_ms", "stream_ms", "total_ms", "rebuilds", "pairs", "steps", "rebuild_ms", "_")
    return dict(zip(keys, out.tolist()))


def md_status(ctx):
    w = C.c_uint32()
    code = lib().md_status(ctx, C.byref(w))
    if code not in (KAMD_OK, KAMD_EDEVICE):
        _check(code, ctx)
    return w.value


def md_clear_status(ctx):
    _check(lib().md_clear_status(ctx), ctx)


def md_destroy(ctx):
    _check(lib().md_destroy(ctx))


# ----------------------------------------------------------- torch wrapper
class System:
    """Replicas of the Kob-Andersen mixture on the current GPU.

    Owns caller-order torch tensors x..az (float64) and img (int32, 3 x n) on
    ``cuda``, and the context's device workspace as a torch uint8 tensor of
    md_workspace_size bytes, which it replaces by a larger one when a call
    reports KAMD_ENOMEM (a longer list after a skin change, an autotuner
    candidate or a healed list overflow) and then repeats the call.
    """

    def __init__(self, replicas, precision="fp64", dt=0.005, skin=0.3, init="given",
                 positions=None, velocities=None, min_dist=0.8, cell_div=1, list_capacity=0.0,
                 auto_sync=True, model=None, device="cuda", dim=3, pe_unshifted=False, sample_every=0,
                 sample_capacity=0, msd_slots=0, own_workspace=True):
        import torch
        self.torch = torch
        self.reps = make_replicas(replicas)
        self.n_rep = len(self.reps)
        self.n_total = sum(r.n for r in self.reps)
        self.offsets = [r.offset for r in self.reps]
        mode = {"given": INIT_GIVEN, "rsa": INIT_RSA, "lattice": INIT_LATTICE}[init]
        self.cfg = make_config(precision, dt, skin, mode, min_dist, cell_div, list_capacity,
                               1 if auto_sync else 0, model, dim, pe_unshifted, sample_every, sample_capacity,
                               msd_slots)
        n = self.n_total
        # a dedicated stream: graph capture is not allowed on the legacy null
        # stream, and every allocation below is ordered on it
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            f64 = dict(dtype=torch.float64, device=device)
            self.t = {k: torch.zeros(n, **f64) for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")}
            self.img = torch.zeros((3, n), dtype=torch.int32, device=device)
            if positions is not None:
                for k, v in zip(("x", "y", "z"), positions):
                    self.t[k].copy_(torch.as_tensor(np.asarray(v, np.float64)))
            if velocities is not None:
                for k, v in zip(("vx", "vy", "vz"), velocities):
                    self.t[k].copy_(torch.as_tensor(np.asarray(v, np.float64)))
        st = State()
        for k, v in self.t.items():
            setattr(st, k, v.data_ptr())
        st.img = self.img.data_ptr()
        self.state = st
        self.device = device
        # room for the list at no less than the default capacity, so that a
        # list that outgrows a smaller list_capacity heals in place
        roomy = make_config(precision, dt, skin, mode, min_dist, cell_div, max(list_capacity, 1.6),
                            1, model, dim, pe_unshifted, sample_every, sample_capacity, msd_slots)
        self.ws_bytes = max(md_workspace_size(self.cfg, self.reps), md_workspace_size(roomy, self.reps))
        self.ws = None
        if own_workspace:
            with torch.cuda.stream(self.stream):
                self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stream.synchronize()
        self.ctx = None
        # own_workspace False: the library allocates (and grows) its own
        self.ctx = md_init(self.cfg, self.reps, st, self.stream.cuda_stream,
                           self.ws.data_ptr() if own_workspace else 0, self.ws_bytes if own_workspace else 0)

    def grow_workspace(self):
        """Move the context into a workspace of md_workspace_needed bytes."""
        need = md_workspace_needed(self.ctx)
        with self.torch.cuda.stream(self.stream):
            ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        md_set_workspace(self.ctx, ws.data_ptr(), need)
        self.ws, self.ws_bytes = ws, need

    def call(self, fn, *args):
        """fn(ctx, *args), repeated once in a larger workspace after KAMD_ENOMEM."""
        try:
            return fn(self.ctx, *args)
        except KamdError as e:
            if e.code != KAMD_ENOMEM:
                raise
            self.grow_workspace()
            return fn(self.ctx, *args)

    def _zeros(self, shape, dtype):
        with self.torch.cuda.stream(self.stream):
            return self.torch.zeros(shape, dtype=dtype, device="cuda")

    def _host(self, t):
        with self.torch.cuda.stream(self.stream):
            return t.cpu().numpy()

    # -- thin methods
    def forces(self, energy=False):
        if energy:
            obs = self._zeros((self.n_rep, 2), self.torch.float64)
            self.call(md_forces, F_FORCE | F_ENERGY | F_VIRIAL, obs.data_ptr())
            return self._host(obs)
        self.call(md_forces, F_FORCE)
        return None

    def step_nve(self, n):
        self.call(md_step_nve, n)

    def step_nvt(self, n, mode=NVT_STOCHASTIC, n_reassign=50, tau=0.5):
        self.call(md_step_nvt, n, mode, n_reassign, tau)

    def build_cells(self):
        self.call(md_build_cells)

    def set_list_params(self, skin, cell_div=1):
        self.call(md_set_list_params, skin, cell_div)

    def autotune(self, probe_steps=100):
        return self.call(md_autotune, probe_steps)

    def set_force_kernel(self, windows, wg_size=0):
        md_set_force_kernel(self.ctx, windows, wg_size)

    def capture(self, nsteps, ensemble=0, mode=NVT_STOCHASTIC, n_reassign=50, tau=0.5):
        md_graph_capture(self.ctx, nsteps, ensemble, mode, n_reassign, tau)

    def launch(self):
        md_graph_launch(self.ctx)

    def rdf(self, dr, n_bins, hist=None):
        if hist is None:
            hist = self._zeros((self.n_rep, 3, n_bins), self.torch.int64)
        md_rdf(self.ctx, dr, n_bins, hist.data_ptr())
        return hist

    def msd_set_origin(self, slot=0):
        md_msd(self.ctx, 0, slot)

    def msd(self, slot=0):
        out = self._zeros((self.n_rep, 2), self.torch.float64)
        md_msd(self.ctx, 1, slot, out.data_ptr())
        return self._host(out)

    def van_hove(self, slot, dr, n_bins, hist=None):
        """Self van Hove histogram against MSD origin `slot`: int64 tensor
        [n_rep][2][n_bins] (accumulated into `hist` when given)."""
        if hist is None:
            hist = self._zeros((self.n_rep, 2, n_bins), self.torch.int64)
        md_van_hove(self.ctx, slot, dr, n_bins, hist.data_ptr())
        return hist

    def set_temperature(self, temperatures):
        """Bath temperature per replica (scalar or sequence)."""
        t = np.broadcast_to(np.asarray(temperatures, np.float64), (self.n_rep,)).copy()
        md_set_temperature(self.ctx, t)

    def scale_velocities(self, factors):
        f = np.broadcast_to(np.asarray(factors, np.float64), (self.n_rep,)).copy()
        md_scale_velocities(self.ctx, f)

    def observables(self):
        """Observables of the current state, [n_rep][6] {KE, PE, W, T, E_tot, P}."""
        return md_observables_now(self.ctx, self.n_rep)

    def samples(self, max_rows=None):
        """Rows of the observables ring, [n_rep][rows][6] {step, KE, PE, E_tot, T, W}."""
        cap = self.cfg.sample_capacity or 1024
        return md_observables(self.ctx, self.n_rep, cap if max_rows is None else max_rows)

    def clear_samples(self):
        md_clear_samples(self.ctx)

    def status(self):
        return md_status(self.ctx)

    def clear_status(self):
        md_clear_status(self.ctx)

    def sync(self):
        md_sync(self.ctx)

    def numpy(self, keys=("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az")):
        self.stream.synchronize()
        return {k: self._host(self.t[k]) for k in keys}

    def images(self):
        self.stream.synchronize()
        return self._host(self.img)

    def replica_slice(self, r):
        o = self.offsets[r]
        return slice(o, o + self.reps[r].n)

    def close(self):
        if self.ctx:
            md_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
