"""The exact range of the MIXED_FIXED pair-force rounding, emulated on the host.

The device rounds each scaled pair-force component q = F * 2^26 to an integer
by adding it to M = 1.5 * 2^52 in one binary64 operation and taking the bit
pattern of the sum minus that of M.  That is exact only while |q| < 2^51,
i.e. |F| < 2^25 force units: beyond it the sum leaves the binade [2^52, 2^53)
and the bits no longer count units.  These tests pin that boundary with the
same binary64 arithmetic (numpy adds with one rounding, as the fma does when
the product is exact), and the separation at which a Kob-Andersen pair force
reaches it (Eq. (KAFix)), which is where the library flags a pair.
"""
import numpy as np
import pytest

M = np.float64(1.5 * 2.0 ** 52)
SCALE = 2.0 ** 26


def device_round(force):
    """Integer force units produced by the magic-number rounding."""
    q = np.float64(force) * np.float64(SCALE)      # exact: a power-of-two scale
    s = q + M                                      # the fma's single rounding
    return int(s.view(np.int64)) - int(M.view(np.int64))


@pytest.mark.parametrize("f", [0.0, 1.0, -1.0, 758.67399573, 3.3e7, -3.3e7, 2.0 ** 25 - 1.0])
def test_rounding_is_exact_below_two_to_the_25(f):
    assert device_round(f) == int(np.rint(f * SCALE))


@pytest.mark.parametrize("f", [3.4e7, 5e7, 8e7, -3.4e7, -5e7])
def test_rounding_is_wrong_beyond_two_to_the_25(f):
    # positive values come out too small, negative ones too large in magnitude
    got = device_round(f) / SCALE
    assert got != pytest.approx(f, rel=1e-3)
    if f > 0:
        assert got < f
    else:
        assert got < f


def pair_force(r, eps, sigma):
    """Magnitude of the Kob-Andersen pair force, Eq. (KAFix)."""
    s6 = (sigma / r) ** 6
    return 48.0 * eps * s6 * (s6 - 0.5) / r


@pytest.mark.parametrize("eps,sigma", [(1.0, 1.0), (1.5, 0.8), (0.5, 0.88)])
def test_separation_where_the_range_ends(eps, sigma):
    """The force falls monotonically on (0, 2^(1/6) sigma) and crosses 2^25
    between 0.30 and 0.40 sigma (where exactly depends on eps/sigma).  The
    emulated rounding is exact just outside the crossing and wrong just
    inside it; a pair at 0.40 sigma stays in range for every pair type."""
    lo, hi = 1e-3 * sigma, 2.0 ** (1 / 6) * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if pair_force(mid, eps, sigma) > 2.0 ** 25:
            lo = mid
        else:
            hi = mid
    rlim = hi
    assert 0.30 * sigma < rlim < 0.40 * sigma
    assert pair_force(0.40 * sigma, eps, sigma) < 2.0 ** 25
    # both sides of the crossing round as the emulation says
    assert device_round(pair_force(1.01 * rlim, eps, sigma)) == int(np.rint(pair_force(1.01 * rlim, eps, sigma) * SCALE))
    f_in = pair_force(0.97 * rlim, eps, sigma)
    assert device_round(f_in) != int(np.rint(f_in * SCALE))


def test_aa_pair_at_0345_is_outside_the_range():
    f = pair_force(0.345, 1.0, 1.0)
    assert f > 2.0 ** 25
    assert device_round(f) != int(np.rint(f * SCALE))
