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
