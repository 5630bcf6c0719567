"""Normalisation of the on-device histograms (host side).

lammps_rdf: the table of LAMMPS compute rdf (Sec. VI.A.3) from the same
counts, taken with n_bins = N_bin and dr = r_cut / N_bin: per pair type g and
the coordination number (mean number of partners of the second type within
the bin's outer radius), columns in the order the paper's command requests
them (AA, BB, AB); write_lammps_rdf writes it in the layout of fix ave/time
mode vector.

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


def lammps_rdf(hist, n: int, n_a: int, L: float, r_cut: float, n_meas: int = 1, dim: int = 3):
    """hist: [3][N_bin] counts of one replica (rows AA, AB, BB as md_rdf
    returns them: ordered pairs, so 2 per AA or BB pair and 1 per AB pair),
    accumulated over n_meas measurements with dr = r_cut / N_bin.  Returns an
    [N_bin][8] array: bin number (from 1), r at the bin centre, g_AA, c_AA,
    g_BB, c_BB, g_AB, c_AB.  g_IJ = counts V / (N_I (N_J - [I = J]) v_bin);
    c_IJ = running sum of counts / N_I."""
    h = np.asarray(hist, np.float64) / float(n_meas)
    nbins = h.shape[1]
    r, size = shells(nbins, r_cut / nbins, dim)
    V = float(L) ** dim
    n_b = n - n_a
    out = np.zeros((nbins, 8))
    out[:, 0] = np.arange(1, nbins + 1)
    out[:, 1] = r
    for col, row, ni, nj in ((2, 0, n_a, n_a - 1), (4, 2, n_b, n_b - 1), (6, 1, n_a, n_b)):
        if ni > 0 and nj > 0:
            out[:, col] = h[row] * V / (ni * nj * size)
        if ni > 0:
            out[:, col + 1] = np.cumsum(h[row]) / ni
    return out


def write_lammps_rdf(f, blocks, fix_id: str = "myrdf", compute_id: str = "rdfAABBAB"):
    """Write (step, table) blocks in the layout of fix ave/time mode vector
    over the compute rdf array: three comment lines, then per block a line
    'step rows' and one line per bin with the row number and the columns."""
    f.write(f"# Time-averaged data for fix {fix_id}\n")
    f.write("# TimeStep Number-of-rows\n")
    f.write("# Row " + " ".join(f"c_{compute_id}[{k}]" for k in range(1, 8)) + "\n")
    for step, table in blocks:
        t = np.asarray(table)
        f.write(f"{int(step)} {t.shape[0]}\n")
        for row in t:
            f.write(f"{int(row[0])} " + " ".join(f"{v:.10g}" for v in row[1:]) + "\n")


def energy_drift(rows, window_steps: int = 500):
    """NVE energy drift from sampled rows {step, KE, PE, E_tot, T, W} of one
    replica (md_observables), per 10^4 steps.

    windowed: |<E>_last - <E>_first| / |<E>_first| with <E> the mean of E_tot
    over the first and the last window_steps of the rows, scaled by 10^4 over
    the distance between the two windows' starts; slope: the least-squares
    slope of E_tot against the step, times 10^4, over |<E>|.  Also the drift
    per particle is left to the caller (divide by N).  Returns a dict.
    """
    import numpy as np
    rows = np.asarray(rows)
    step, e = rows[:, 0], rows[:, 3]
    if len(step) < 4:
        return {"windowed": float("nan"), "slope": float("nan"), "steps": 0}
    ds = step[1] - step[0]
    first = e[step < step[0] + window_steps]
    last = e[step > step[-1] - window_steps]
    span = (step[-1] - step[0]) - window_steps + ds
    windowed = abs(last.mean() - first.mean()) / abs(first.mean()) * (1e4 / span) if span > 0 else float("nan")
    slope = np.polyfit(step, e, 1)[0]
    return {"windowed": float(windowed), "slope": float(abs(slope) * 1e4 / abs(e.mean())),
            "steps": int(step[-1] - step[0] + ds), "window_steps": int(window_steps),
            "e_mean": float(e.mean())}
