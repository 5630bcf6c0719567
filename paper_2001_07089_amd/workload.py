"""Seeded synthetic inputs for the Kob-Andersen workloads.

This module draws random numbers and lays out arrays; it contains none of the
method's arithmetic (no forces, integration, thermostat or analysis).  It is
the one module that both the GPU tests and the oracle tests take their inputs
from.

Workload shapes follow the paper's Kob-Andersen mixture (Sec. II.B: 80:20,
number density about 1.2, N = 1000 with L = 9.4 in the paper's examples) and
the scaled-up single-system and replica-batch configurations defined below.  The paper's own configuration files are not available, so every
configuration is generated here from a seed.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

BASE_SEED = 2001070890


def n_a_for(n: int, frac_a: float = 0.8) -> int:
    """Number of A particles of an 80:20 mixture, rounded half up."""
    return int(np.floor(frac_a * n + 0.5))


def box_for(n: int, rho: float) -> float:
    """Cubic box edge for n particles at number density rho."""
    return float((n / rho) ** (1.0 / 3.0))


def lattice_config(n: int, L: float, seed: int, jitter: float = 0.1):
    """Positions on a simple cubic lattice with uniform jitter, random site order.

    n sites are chosen at random from the smallest m^3 >= n lattice with
    spacing L/m; each position gets an independent uniform jitter of
    +-jitter*spacing and is wrapped into [0, L).  Returns x, y, z (float64).
    """
    rng = np.random.default_rng(seed)
    m = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
    while m ** 3 < n:
        m += 1
    a = L / m
    sites = rng.permutation(m ** 3)[:n]
    ix, iy, iz = sites % m, (sites // m) % m, sites // (m * m)
    pos = []
    for k in (ix, iy, iz):
        u = (k + 0.5) * a + rng.uniform(-jitter, jitter, size=n) * a
        u = np.mod(u, L)
        u[u >= L] = 0.0
        pos.append(u.astype(np.float64))
    return pos[0], pos[1], pos[2]


def uniform_config(n: int, L: float, seed: int):
    """Independent uniform positions in [0, L)^3."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, L, size=(3, n))
    p[p >= L] = 0.0
    return p[0].copy(), p[1].copy(), p[2].copy()


def gaussian_velocities(n: int, scale: float, seed: int):
    """Independent normal velocity components with standard deviation `scale`."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, scale, size=(3, n))
    return v[0].copy(), v[1].copy(), v[2].copy()


@dataclass
class Replica:
    n: int
    n_a: int
    box: float
    temperature: float
    seed: int
    rho: float = 1.2


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    dt: float = 0.005
    steps: int = 1000
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_total(self) -> int:
        return sum(r.n for r in self.replicas)


def single(name: str, n: int, rho: float, T: float, cfg_index: int, steps: int,
           description: str = "") -> Workload:
    rep = Replica(n=n, n_a=n_a_for(n), box=box_for(n, rho), temperature=T,
                  seed=BASE_SEED + 1000 * cfg_index, rho=rho)
    return Workload(name=name, replicas=[rep], steps=steps, description=description)


def ka_small() -> Workload:
    """N = 1000 (800 A / 200 B) at density 1.2, T0 = 2.0, 1000 NVE steps."""
    return single("ka_n1000_rho1.2_T2.0_nve", 1000, 1.2, 2.0, 1, 1000)


def ka_planar(n: int = 1000, T: float = 0.4) -> Workload:
    """The planar KA variant of the appendix exercise: 65:35 mixture at
    N/L^2 = 1.204 (L = 28.82 for N = 1000), z = vz = 0, T < 0.5."""
    L = float(np.sqrt(n / 1.204))
    rep = Replica(n=n, n_a=n_a_for(n, 0.65), box=L, temperature=T, seed=BASE_SEED + 7000, rho=1.204)
    return Workload(name=f"ka2d_n{n}_rho1.204_T{T}", replicas=[rep], steps=1000)


def planar_lattice_config(n: int, L: float, seed: int, jitter: float = 0.05):
    """Positions on a square lattice in the plane z = 0 with uniform jitter,
    random site order (x, y, z with z = 0)."""
    m = int(np.ceil(np.sqrt(n) - 1e-9))
    while m * m < n:
        m += 1
    a = L / m
    rng = np.random.default_rng(seed)
    sites = rng.permutation(m * m)[:n]
    x = (sites % m + 0.5 + rng.uniform(-jitter, jitter, n)) * a
    y = (sites // m + 0.5 + rng.uniform(-jitter, jitter, n)) * a
    return np.mod(x, L), np.mod(y, L), np.zeros(n)


def ka_medium() -> Workload:
    """N = 32,000 (25,600 A / 6,400 B) at density 1.2, T = 0.5."""
    return single("ka_n32000_rho1.2_T0.5", 32000, 1.2, 0.5, 2, 10000)


def ka_large() -> Workload:
    """N = 1,048,576 (838,861 A / 209,715 B) at density 1.2, T = 0.45, 5000 NVE steps."""
    return single("ka_n1048576_rho1.2_T0.45_nve", 1 << 20, 1.2, 0.45, 3, 5000)


def ka_batch_small(n_rep: int = 256) -> Workload:
    """n_rep replicas, N uniform on [250, 8000], density 1.2, T evenly on [0.45, 2.0]."""
    rng = np.random.default_rng(BASE_SEED + 4000)
    ns = rng.integers(250, 8001, size=n_rep)
    reps = []
    for r in range(n_rep):
        n = int(ns[r])
        T = 0.45 + (2.0 - 0.45) * r / max(1, n_rep - 1)
        reps.append(Replica(n=n, n_a=n_a_for(n), box=box_for(n, 1.2), temperature=T,
                            seed=BASE_SEED + 4000 + r, rho=1.2))
    return Workload(name=f"ka_batch{n_rep}_n250-8000_rho1.2_T0.45-2.0", replicas=reps, steps=1000)


def ka_batch_large(n_rep: int = 64) -> Workload:
    """n_rep replicas, N uniform on [50,000, 500,000], density in {1.1, 1.2, 1.3},
    T uniform on [0.45, 1.0]."""
    rng = np.random.default_rng(BASE_SEED + 5000)
    ns = rng.integers(50000, 500001, size=n_rep)
    rhos = rng.choice(np.array([1.1, 1.2, 1.3]), size=n_rep)
    Ts = rng.uniform(0.45, 1.0, size=n_rep)
    reps = []
    for r in range(n_rep):
        n = int(ns[r])
        rho = float(rhos[r])
        reps.append(Replica(n=n, n_a=n_a_for(n), box=box_for(n, rho), temperature=float(Ts[r]),
                            seed=BASE_SEED + 5000 + r, rho=rho))
    return Workload(name=f"ka_batch{n_rep}_n50k-500k_rho1.1-1.3_T0.45-1.0", replicas=reps,
                    steps=2000)
