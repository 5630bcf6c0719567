"""Host normalisation of the histograms against the oracle's normalisation
and against integrals that the definitions fix."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import analysis


@pytest.mark.parametrize("dim", [3, 2])
def test_rdf_normalisation_matches_oracle(dim):
    rng = np.random.default_rng(5)
    h = rng.integers(0, 5000, size=(3, 120)).astype(np.uint64)
    n, na, L, dr, nm = 1000, 650 if dim == 2 else 800, 28.82 if dim == 2 else 9.41, 0.04, 7
    r, g = analysis.rdf(h, n, na, L, dr, nm, dim)
    r0, g0 = O.rdf_normalize(h, n, na, L, dr, nm, dim=dim)
    assert np.allclose(r, r0, rtol=1e-14) and np.allclose(g, g0, rtol=1e-12)


def test_van_hove_normalisation_integrates_to_one():
    """sum_b G_s(r_b) * shell_b = 1 for counts that hold every particle."""
    n, na, dr = 1000, 800, 0.01
    rng = np.random.default_rng(9)
    h = np.zeros((2, 300))
    np.add.at(h[0], rng.integers(0, 300, na), 1)
    np.add.at(h[1], rng.integers(0, 300, n - na), 1)
    for dim in (3, 2):
        r, G = analysis.van_hove_self(h, n, na, dr, dim)
        _, size = analysis.shells(300, dr, dim)
        assert np.allclose((G * size).sum(axis=1), 1.0, rtol=1e-12)
    assert analysis.shells(1, 1.0, 3)[1][0] == pytest.approx(4 * math.pi / 3)
    assert analysis.shells(1, 1.0, 2)[1][0] == pytest.approx(math.pi)


def test_energy_drift_windowed_and_slope():
    """A linear energy ramp of known slope: both definitions return it."""
    import numpy as np
    from paper_2001_07089_amd import analysis
    steps = np.arange(10, 10001, 10, dtype=float)
    e = -6000.0 * (1.0 + 2e-9 * steps)            # relative drift 2e-5 per 10^4 steps
    rows = np.zeros((steps.size, 6))
    rows[:, 0], rows[:, 3] = steps, e
    out = analysis.energy_drift(rows, 500)
    assert abs(out["windowed"] - 2e-5) < 1e-7
    assert abs(out["slope"] - 2e-5) < 1e-7
    rows[:, 3] = -6000.0 + 0.01 * np.sin(steps)   # fluctuation only: no drift
    assert analysis.energy_drift(rows, 500)["slope"] < 1e-6
