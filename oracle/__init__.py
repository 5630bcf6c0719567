"""CPU oracle for the Kob-Andersen binary Lennard-Jones MD method (arXiv:2001.07089).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It is a plain,
slow, FP64 implementation of what the paper defines (see ``ka_oracle.c`` for
the per-function citations) and shares no code with the GPU library
``paper_2001_07089_amd``; neither imports the other.

Arrays are numpy float64 / int32 in the caller's particle order: the A block
(indices 0..na-1) first, then the B block.  Image counters are int32 arrays of
shape (3, n).

Each function is pinned by tests/test_oracle.py to something other than
itself (closed forms, invariants, brute force, library routines); the absolute
energy level of a KA liquid and the shapes of its RDF and MSD curves are
"parity unpinned" (checked only for the excluded core and the uniform limit
of g(r)).
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_LIB = None

# Kob-Andersen parameters (Sec. II.B): pair order AA, AB, BB.
KA_EPS = (1.0, 1.5, 0.5)
KA_SIGMA = (1.0, 0.8, 0.88)
KA_RC_FACTOR = 2.5


class Model(C.Structure):
    _fields_ = [("eps", C.c_double * 3), ("sigma", C.c_double * 3), ("rc_factor", C.c_double)]


def model(eps=KA_EPS, sigma=KA_SIGMA, rc_factor=KA_RC_FACTOR) -> Model:
    m = Model()
    for p in range(3):
        m.eps[p] = float(eps[p])
        m.sigma[p] = float(sigma[p])
    m.rc_factor = float(rc_factor)
    return m


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_U32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        MP = C.POINTER(Model)
        L.ora_pair_force.argtypes = [MP, C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.ora_pair_force.restype = C.c_double
        for name in ("ora_forces_brute", "ora_forces_cell"):
            f = getattr(L, name)
            f.argtypes = [MP, C.c_int, C.c_int, C.c_double, _D, _D, _D, _D, _D, _D,
                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
            f.restype = None
        L.ora_min_distance.argtypes = [C.c_int, C.c_double, _D, _D, _D]
        L.ora_min_distance.restype = C.c_double
        L.ora_kinetic.argtypes = [C.c_int, _D, _D, _D]
        L.ora_kinetic.restype = C.c_double
        L.ora_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.ora_philox4x32_10.restype = None
        L.ora_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _D]
        L.ora_gauss3.restype = None
        L.ora_mb_velocities.argtypes = [C.c_int, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32,
                                        C.c_void_p, _D, _D, _D]
        L.ora_mb_velocities.restype = None
        L.ora_mb_velocities_d.argtypes = [C.c_int, C.c_int, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32,
                                          C.c_void_p, _D, _D, _D]
        L.ora_mb_velocities_d.restype = None
        L.ora_run.argtypes = [MP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                              C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _I32,
                              C.c_int, C.c_double, C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p]
        L.ora_run.restype = None
        L.ora_run_nh.argtypes = [MP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                 C.c_double, C.c_double, C.c_int,
                                 _D, _D, _D, _D, _D, _D, _D, _D, _D, _I32, _D, C.c_void_p]
        L.ora_run_nh.restype = None
        L.ora_rdf_hist.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D, _D, C.c_double,
                                   C.c_int, _U64]
        L.ora_rdf_hist.restype = None
        L.ora_msd.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D, _D, _I32, _D, _D, _D, _D]
        L.ora_msd.restype = None
        L.ora_van_hove_self.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D, _D, _I32, _D, _D, _D,
                                        C.c_double, C.c_int, _U64]
        L.ora_van_hove_self.restype = None
        L.ora_log_schedule.argtypes = [C.c_int, C.c_double, C.c_int, _I32, C.c_int]
        L.ora_log_schedule.restype = C.c_int
        L.ora_num_threads.argtypes = []
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int]
        L.ora_set_num_threads.restype = None
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (n < 1: all processors)."""
    lib().ora_set_num_threads(int(n))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def pair_force(p: int, r2: float, m: Model = None):
    """Closed form of one pair (Eqs. (KAFix),(VshiftedKALJ)): returns (f, V_shifted)."""
    m = m or model()
    v = C.c_double()
    f = lib().ora_pair_force(C.byref(m), int(p), float(r2), C.byref(v))
    return f, v.value


def forces(x, y, z, na: int, L: float, method: str = "cell", m: Model = None):
    """Forces (= accelerations, m = 1), total shifted PE and virial W.

    method: "brute" (O(N^2) half loop with Newton's third law) or "cell".
    Returns (fx, fy, fz, pe, w).
    """
    m = m or model()
    x, y, z = _c(x), _c(y), _c(z)
    n = x.size
    fx, fy, fz = np.empty(n), np.empty(n), np.empty(n)
    pe, w = C.c_double(), C.c_double()
    fn = lib().ora_forces_brute if method == "brute" else lib().ora_forces_cell
    fn(C.byref(m), n, int(na), float(L), x, y, z, fx, fy, fz, C.byref(pe), C.byref(w))
    return fx, fy, fz, pe.value, w.value


def min_distance(x, y, z, L):
    x, y, z = _c(x), _c(y), _c(z)
    return lib().ora_min_distance(x.size, float(L), x, y, z)


def kinetic(vx, vy, vz):
    vx, vy, vz = _c(vx), _c(vy), _c(vz)
    return lib().ora_kinetic(vx.size, vx, vy, vz)


def philox4x32_10(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def gauss3(seed: int, rep: int, tag: int, pid: int):
    g = np.zeros(3)
    lib().ora_gauss3(int(seed), int(rep), int(tag), int(pid), g)
    return g


def mb_velocities(n: int, T: float, seed: int, rep: int = 0, tag: int = 0, ids=None, dim: int = 3):
    """Maxwell-Boltzmann flow chart of Sec. II.E.1 with Philox Gaussians
    (dim 2: planar, vz = 0, sum v^2 = 2 N T)."""
    vx, vy, vz = np.empty(n), np.empty(n), np.empty(n)
    ids_arr = None if ids is None else _c(ids, np.int32)
    lib().ora_mb_velocities_d(int(dim), int(n), float(T), int(seed), int(rep), int(tag),
                              None if ids_arr is None else ids_arr.ctypes.data, vx, vy, vz)
    return vx, vy, vz


class State:
    """Mutable FP64 state of one system, in caller order."""

    def __init__(self, x, y, z, vx, vy, vz, na, L, img=None):
        self.x, self.y, self.z = _c(x).copy(), _c(y).copy(), _c(z).copy()
        self.vx, self.vy, self.vz = _c(vx).copy(), _c(vy).copy(), _c(vz).copy()
        self.n = self.x.size
        self.na = int(na)
        self.L = float(L)
        self.img = np.zeros((3, self.n), np.int32) if img is None else _c(img, np.int32).copy()
        self.ax = np.zeros(self.n)
        self.ay = np.zeros(self.n)
        self.az = np.zeros(self.n)
        self.xi = 0.0
        self.lns = 0.0

    def copy(self):
        s = State(self.x, self.y, self.z, self.vx, self.vy, self.vz, self.na, self.L, self.img)
        s.ax, s.ay, s.az = self.ax.copy(), self.ay.copy(), self.az.copy()
        s.xi, s.lns = self.xi, self.lns
        return s

    def compute_forces(self, method="cell", m=None):
        self.ax, self.ay, self.az, pe, w = forces(self.x, self.y, self.z, self.na, self.L, method, m)
        return pe, w


def run(st: State, dt: float, nsteps: int, method: str = "cell", m: Model = None,
        step0: int = 0, nb: int = 0, T: float = 0.0, seed: int = 0, rep: int = 0, ids=None, dim: int = 3):
    """Velocity-Verlet NVE steps (optionally with the stochastic bath every nb steps).

    st.ax.. must hold the forces of the entry positions.  Returns an array
    (nsteps, 3) of {KE, PE, W} after each step.
    """
    m = m or model()
    e = np.zeros((nsteps, 3))
    ids_arr = None if ids is None else _c(ids, np.int32)
    lib().ora_run(C.byref(m), 1 if method == "cell" else 0, int(dim), st.n, st.na, st.L, float(dt),
                  int(nsteps), int(step0), st.x, st.y, st.z, st.vx, st.vy, st.vz,
                  st.ax, st.ay, st.az, st.img, int(nb), float(T), int(seed), int(rep),
                  None if ids_arr is None else ids_arr.ctypes.data, e.ctypes.data)
    return e


def run_nh(st: State, dt: float, nsteps: int, T: float, Q: float, method: str = "cell",
           m: Model = None, exact_solve: bool = False, dim: int = 3):
    """Nose-Hoover steps (Fox-Andersen scheme of Appendix B).

    Returns (nsteps, 5) of {KE, PE, W, xi, ln s} after each step.
    """
    m = m or model()
    e = np.zeros((nsteps, 5))
    nh = np.array([st.xi, st.lns])
    lib().ora_run_nh(C.byref(m), 1 if method == "cell" else 0, int(dim), st.n, st.na, st.L, float(dt),
                     int(nsteps), float(T), float(Q), 1 if exact_solve else 0,
                     st.x, st.y, st.z, st.vx, st.vy, st.vz, st.ax, st.ay, st.az, st.img,
                     nh, e.ctypes.data)
    st.xi, st.lns = float(nh[0]), float(nh[1])
    return e


def nh_conserved(e_row, n, T, Q, dim: int = 3):
    """Eq. (HNosetilde): KE + PE + Q xi^2 / 2 + X T ln s with X = d N."""
    ke, pe, _, xi, lns = e_row
    return ke + pe + 0.5 * Q * xi * xi + float(dim) * n * T * lns


def rdf_hist(x, y, z, na, L, dr, nbins, hist=None):
    """Pair-distance histogram (Sec. VI.A.1); rows AA, AB, BB; uint64."""
    x, y, z = _c(x), _c(y), _c(z)
    h = np.zeros((3, nbins), np.uint64) if hist is None else hist
    lib().ora_rdf_hist(x.size, int(na), float(L), x, y, z, float(dr), int(nbins), h)
    return h


def rdf_normalize(hist, n, na, L, dr, nmeas, dim: int = 3):
    """g_AA, g_AB, g_BB at bin mid-points (Eqs. (gAA),(gAB); normalisation of Sec. VI.A.1).

    Shell volume (4 pi / 3)(r_out^3 - r_in^3) and V = L^3; for the planar
    system (dim 2, the appendix exercise) the shell area pi (r_out^2 - r_in^2)
    and V = L^2.  nmeas measurements.  Returns (r_mid, g), rows AA, AB, BB.
    """
    nb = n - na
    nbins = hist.shape[1]
    g = np.zeros((3, nbins))
    rmid = np.zeros(nbins)
    V = L ** dim
    for b in range(nbins):
        rin = b * dr
        rout = rin + dr
        if dim == 2:
            shell = math.pi * (rout ** 2 - rin ** 2)
        else:
            shell = (4.0 * math.pi / 3.0) * (rout ** 3 - rin ** 3)
        g[0, b] = (V / (na * (na - 1))) * float(hist[0, b]) / (shell * nmeas) if na > 1 else 0.0
        g[1, b] = (V / (na * nb)) * float(hist[1, b]) / (shell * nmeas) if na > 0 and nb > 0 else 0.0
        g[2, b] = (V / (nb * (nb - 1))) * float(hist[2, b]) / (shell * nmeas) if nb > 1 else 0.0
        rmid[b] = rin + 0.5 * dr
    return rmid, g


def pe_lj_cut(x, y, z, na, L, m: Model = None):
    """Potential energy of the truncated pair potential without the shift:
    the sum over pairs closer than r_c(ab) of Eq. (VKALJ) alone, i.e. the
    constant V_ab(r_c) of Eq. (VshiftedKALJ) left out.  This is the energy
    LAMMPS pair style lj/cut reports (Sec. IV.B notes that it omits that term);
    the forces are the same.  Plain brute force over all pairs, minimum image
    by rounding (Sec. II.C), FP64."""
    m = m or model()
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    n = x.size
    typ = (np.arange(n) >= na).astype(np.int64)
    eps = np.array(m.eps[:], np.float64)
    sig = np.array(m.sigma[:], np.float64)
    e = 0.0
    for i in range(n - 1):
        dx = x[i + 1:] - x[i]
        dy = y[i + 1:] - y[i]
        dz = z[i + 1:] - z[i]
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        dz -= L * np.round(dz / L)
        r2 = dx * dx + dy * dy + dz * dz
        p = typ[i] + typ[i + 1:]
        rc = m.rc_factor * sig[p]
        sel = r2 < rc * rc
        sr6 = (sig[p][sel] ** 2 / r2[sel]) ** 3
        e += float(np.sum(4.0 * eps[p][sel] * (sr6 * sr6 - sr6)))
    return e


def lammps_rdf_table(hist, n, na, L, rcut, nbins, nmeas=1):
    """The table of LAMMPS compute rdf (Sec. VI.A.3): nbins bins of width
    rcut / nbins from 0, and per pair type I-J (order AA, BB, AB as in the
    paper's command) g_IJ and the coordination number c_IJ, the mean number of
    J particles within the bin's outer radius of an I particle.

    hist: [3][nbins] pair-distance counts over nmeas measurements with rows AA
    (2 per pair), AB (1 per pair), BB (2 per pair), i.e. ordered I-J pairs.
    g_IJ(bin) = counts / (nmeas N_I (N_J - [I = J]) v_bin / V), with v_bin the
    shell volume; c_IJ(bin) = sum over bins <= bin of counts / (nmeas N_I).
    Returns rows [bin number (1-based), r at the bin centre, g_AA, c_AA, g_BB,
    c_BB, g_AB, c_AB]."""
    nb = n - na
    dr = rcut / nbins
    V = L ** 3
    rows = []
    # (hist row, N_I, N_J, same type)
    pairs = ((0, na, na, True), (2, nb, nb, True), (1, na, nb, False))
    cum = [0.0, 0.0, 0.0]
    for b in range(nbins):
        rin, rout = b * dr, (b + 1) * dr
        shell = (4.0 * math.pi / 3.0) * (rout ** 3 - rin ** 3)
        row = [b + 1, rin + 0.5 * dr]
        for k, (h, ni, nj, same) in enumerate(pairs):
            cnt = float(hist[h][b]) / nmeas
            njj = nj - 1 if same else nj
            g = cnt / (ni * njj * shell / V) if ni > 0 and njj > 0 else 0.0
            cum[k] += cnt / ni if ni > 0 else 0.0
            row += [g, cum[k]]
        rows.append(row)
    return np.array(rows, np.float64)


def msd(x, y, z, img, na, L, x0u, y0u, z0u):
    """Per-species MSD of unwrapped positions against an unwrapped origin."""
    out = np.zeros(2)
    x, y, z = _c(x), _c(y), _c(z)
    lib().ora_msd(x.size, int(na), float(L), x, y, z, _c(img, np.int32), _c(x0u), _c(y0u),
                  _c(z0u), out)
    return out


def van_hove_self(x, y, z, img, na, L, x0u, y0u, z0u, dr, nbins):
    """Self van Hove histogram per species ([2][nbins] uint64) of the unwrapped
    displacements against an unwrapped origin."""
    out = np.zeros((2, int(nbins)), np.uint64)
    x, y, z = _c(x), _c(y), _c(z)
    lib().ora_van_hove_self(x.size, int(na), float(L), x, y, z, _c(img, np.int32), _c(x0u), _c(y0u), _c(z0u),
                            float(dr), int(nbins), out)
    return out


def unwrapped(x, y, z, img, L):
    img = np.asarray(img)
    return (np.asarray(x) + img[0] * L, np.asarray(y) + img[1] * L, np.asarray(z) + img[2] * L)


def log_schedule(nmd: int, t0: float = 1.0, kmax: int = 60):
    """Log-spaced measurement steps of Sec. VI.B.1."""
    buf = np.zeros(max(16, 4 * kmax + 16), np.int32)
    n = lib().ora_log_schedule(int(nmd), float(t0), int(kmax), buf, buf.size)
    return buf[:min(n, buf.size)].copy()
