"""Pairs placed at the cutoff and pairs too close for the fixed-point range.

Cutoff (Eq. (KAFix), strict r < r_c = 2.5 sigma_ab): two-particle replicas of
each pair type (AA, AB, BB) in several box sizes, at r = r_c (1 - 2^-20),
exactly r_c and r_c (1 + 2^-20), along an axis, along a diagonal and across
the periodic boundary.  FP64 forces and energies must equal the oracle's strict
test to 1e-12 (exactly zero outside); the mixed precisions classify every
pair 2^-20 away from r_c as the oracle does and give its force to 1e-5, and at
exactly r_c (where their FP32 test may go either way, within ~4e-7 of r_c)
give either zero or the force just inside.

Fixed-point range: MIXED_FIXED rounds each pair force component to 2^-26
units exactly only while |F| < 2^25.  A pair closer than the separation where
that bound is reached (found here by bisection on the closed-form force of
each pair type) sets KAMD_DEV_FORCE_RANGE; a pair outside it does not, and its
force matches the oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import md

pytestmark = pytest.mark.gpu

SIG = {0: 1.0, 1: 0.8, 2: 0.88}     # AA, AB, BB (Sec. II.B)
NA = {0: 2, 1: 1, 2: 0}             # n_a of a two-particle replica of that pair type
BOXES = (5.5, 9.41, 13.7)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rc_of(p):
    return 2.5 * SIG[p]  # the library and the oracle form r_c = rc_factor * sigma in binary64


def cases():
    """(pair type, box, label, x, y, z) for every crafted pair."""
    out = []
    eps = 2.0 ** -20
    for p in (0, 1, 2):
        rc = rc_of(p)
        for L in BOXES:
            # exactly representable along x: 1.0 and 1.0 + r_c differ by r_c exactly when
            # the sum is exact (checked), else the pair sits within one ulp of r_c and the
            # oracle's strict test on the same inputs decides
            x0 = 1.0
            for lab, f in (("in", 1.0 - eps), ("at", 1.0), ("out", 1.0 + eps)):
                r = rc * f
                out.append((p, L, "axis-" + lab, np.array([x0, x0 + r]), np.array([2.0, 2.0]), np.array([3.0, 3.0])))
            u = np.array([1.0, 2.0, 2.0]) / 3.0
            for lab, f in (("in", 1.0 - eps), ("out", 1.0 + eps)):
                r = rc * f
                a = np.array([0.3 * L, 0.25 * L, 0.2 * L])
                b = a + r * u
                out.append((p, L, "diag-" + lab, np.array([a[0], b[0]]), np.array([a[1], b[1]]), np.array([a[2], b[2]])))
            for lab, f in (("in", 1.0 - eps), ("out", 1.0 + eps)):
                r = rc * f
                xa = L - 0.4 * rc
                xb = (xa + r) - L  # the partner sits across the boundary
                out.append((p, L, "wrap-" + lab, np.array([xa, xb]), np.array([1.0, 1.0]), np.array([1.5, 1.5])))
    return out


def build(sel, prec):
    reps, xs, ys, zs = [], [], [], []
    for k, (p, L, lab, x, y, z) in enumerate(sel):
        reps.append((2, NA[p], L, 1.0, 500 + k))
        xs.append(x)
        ys.append(y)
        zs.append(z)
    zero = [np.zeros(2 * len(sel))] * 3
    return md.System(reps, precision=prec, positions=(np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)),
                     velocities=zero)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_fixed"])
def test_pairs_at_the_cutoff(prec):
    sel = cases()
    log(f"case cutoff edges {prec}: {len(sel)} two-particle replicas")
    s = build(sel, prec)
    obs = s.forces(energy=True)
    a = s.numpy()
    assert s.status() == 0
    n_in = n_out = 0
    for k, (p, L, lab, x, y, z) in enumerate(sel):
        fx, fy, fz, pe, w = O.forces(x, y, z, NA[p], L, "brute")
        ref = np.array([fx[0], fy[0], fz[0]])
        got = np.array([a["ax"][2 * k], a["ay"][2 * k], a["az"][2 * k]])
        got_j = np.array([a["ax"][2 * k + 1], a["ay"][2 * k + 1], a["az"][2 * k + 1]])
        inside = np.any(ref != 0.0)
        n_in += inside
        n_out += not inside
        tag = (prec, p, L, lab)
        if prec == "fp64":
            if inside:
                assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), tag
                assert obs[k, 0] == pytest.approx(pe, rel=1e-12, abs=1e-15), tag
            else:
                assert np.all(got == 0.0) and np.all(got_j == 0.0), tag
                assert obs[k, 0] == 0.0 and pe == 0.0, tag
        elif lab == "axis-at":
            # either classification is a correct FP32 answer this close to r_c
            rin = rc_of(p) * (1.0 - 2.0 ** -30)
            fin = O.pair_force(p, rin * rin)[0] * rin
            mag = np.linalg.norm(got)
            assert mag == 0.0 or abs(mag - abs(fin)) <= 1e-5 * abs(fin), (tag, mag, fin)
        else:
            if inside:
                assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), (tag, got, ref)
                # the shifted pair energy V(r) - V(r_c) is ~1e-7 here: its FP32
                # terms cancel, so the bound is absolute (a few FP32 ulps of
                # V(r_c) ~ 0.02 eps)
                assert abs(obs[k, 0] - pe) <= 1e-7, (tag, obs[k, 0], pe)
            else:
                assert np.all(got == 0.0), (tag, got)
                assert obs[k, 0] == 0.0, tag
        # Newton's third law holds for every precision (exactly for the
        # fixed-point sums and FP64's single pair)
        if prec != "mixed":
            assert np.all(got == -got_j), tag
    assert n_in > 0 and n_out > 0
    s.close()


def two_close(p, r, prec, L=9.41):
    x = np.array([2.0, 2.0 + r])
    y = np.array([4.0, 4.0])
    z = np.array([5.0, 5.0])
    return md.System([(2, NA[p], L, 1.0, 77)], precision=prec, positions=(x, y, z),
                     velocities=[np.zeros(2)] * 3), (x, y, z)


EPS = {0: 1.0, 1: 1.5, 2: 0.5}


def range_limit(p):
    """Separation at which the pair force of type p reaches 2^25 (Eq. (KAFix))."""
    def f(r):
        s6 = (SIG[p] / r) ** 6
        return 48.0 * EPS[p] * s6 * (s6 - 0.5) / r
    lo, hi = 1e-3 * SIG[p], 2.0 ** (1 / 6) * SIG[p]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 2.0 ** 25 else (lo, mid)
    return hi


@pytest.mark.parametrize("p", [0, 1, 2])
def test_fixed_point_range_is_flagged_per_pair(p):
    """3% inside the separation where |F| reaches 2^25 (the force is then
    1.5 times the bound) -> the range bit; 5% outside it -> no bit, and the
    force equals the oracle's."""
    rlim = range_limit(p)
    for factor, expect_bit in ((0.97, True), (1.05, False)):
        r = factor * rlim
        s, (x, y, z) = two_close(p, r, "mixed_fixed")
        word = s.status()
        log(f"case range p={p} r={r:.4f}: word 0x{word:x}")
        assert bool(word & md.DEV_FORCE_RANGE) == expect_bit, (p, r, word)
        if not expect_bit:
            a = s.numpy()
            fx, _, _, _, _ = O.forces(x, y, z, NA[p], 9.41, "brute")
            assert a["ax"][0] == pytest.approx(fx[0], rel=1e-5)
            assert a["ax"][1] == -a["ax"][0]
        s.close()
    # the other precisions have no such bound: no bit, forces as the oracle's
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        r = 0.97 * rlim
        s, (x, y, z) = two_close(p, r, prec)
        assert s.status() == 0
        fx, _, _, _, _ = O.forces(x, y, z, NA[p], 9.41, "brute")
        assert s.numpy()["ax"][0] == pytest.approx(fx[0], rel=tol)
        s.close()
