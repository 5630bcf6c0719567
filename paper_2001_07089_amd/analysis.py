"""Normalisation of the on-device histograms (host side).

rdf: g_ab(r) from the pair-distance counts of ``md_rdf`` (Eqs. (gAA),
(gAB) and the normalisation described in Sec. VI.A.1): the counts of bin b
(AA and BB rows hold 2 per pair, AB 1) divided by the number of measurements,
by the shell volume (4 pi / 3)(r_out^3 - r_in^3) -- the shell area
pi (r_out^2 - r_in^2) for the planar system -- and by N_a (N_a - 1) / V
(same species) or N_a N_b / V (AB), with V = L^d.

van Hove: G_s(r, t) from the self-displacement counts of ``md_van_hove``,
divided by N_a and by the shell volume (area), so that its integral over
space is 1.
"""
import math

import numpy as np


def shells(n_bins: int, dr: float, dim: int = 3):
    """(r_mid, shell volume or area) for bins [b dr, (b+1) dr)."""
    edges = np.arange(n_bins + 1, dtype=np.float64) * dr
    if dim == 2:
        size = math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    else:
        size = (4.0 * math.pi / 3.0) * (edges[1:] ** 3 - edges[:-1] ** 3)
    return 0.5 * (edges[1:] + edges[:-1]), size


def rdf(hist, n: int, n_a: int, L: float, dr: float, n_meas: int = 1, dim: int = 3):
    """hist: [3][n_bins] counts of one replica (rows AA, AB, BB).  Returns
    (r_mid, g) with g rows AA, AB, BB (zero where a species pair is empty)."""
    h = np.asarray(hist, np.float64)
    r, size = shells(h.shape[1], dr, dim)
    V = float(L) ** dim
    n_b = n - n_a
    pairs = np.array([n_a * (n_a - 1), n_a * n_b, n_b * (n_b - 1)], np.float64)
    g = np.zeros_like(h)
    ok = pairs > 0
    g[ok] = (V / pairs[ok, None]) * h[ok] / (size[None, :] * n_meas)
    return r, g


def van_hove_self(hist, n: int, n_a: int, dr: float, dim: int = 3):
    """hist: [2][n_bins] counts of one replica (rows A, B).  Returns (r_mid,
    G_s) with rows A, B."""
    h = np.asarray(hist, np.float64)
    r, size = shells(h.shape[1], dr, dim)
    counts = np.array([n_a, n - n_a], np.float64)
    G = np.zeros_like(h)
    ok = counts > 0
    G[ok] = h[ok] / (counts[ok, None] * size[None, :])
    return r, G
