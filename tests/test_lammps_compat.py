"""LAMMPS compatibility helpers (host side, no GPU): data and dump files, and
the compute-rdf table with coordination numbers built from pair counts."""
import io
import math

import numpy as np
import pytest

import oracle as O
from paper_2001_07089_amd import analysis as A
from paper_2001_07089_amd import lammps_io as LIO
from paper_2001_07089_amd import workload as W


def _config(n=300, seed=4):
    L = (n / 1.2) ** (1.0 / 3.0)
    x, y, z = W.lattice_config(n, L, seed, 0.2)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n))
    img = rng.integers(-3, 4, size=(3, n)).astype(np.int32)
    return L, W.n_a_for(n), (x, y, z), v, img


def test_data_file_round_trip_is_exact():
    L, na, (x, y, z), v, img = _config()
    buf = io.StringIO()
    LIO.write_data(buf, x, y, z, na, L, *v, img=img)
    text = buf.getvalue()
    assert f"{x.size} atoms" in text and "2 atom types" in text and "Velocities" in text
    got = LIO.read_data(io.StringIO(text))
    assert got["n"] == x.size and got["n_a"] == na and got["L"] == L
    assert np.array_equal(got["ids"], np.arange(1, x.size + 1))
    for k, a in zip(("x", "y", "z", "vx", "vy", "vz"), (x, y, z, *v)):
        assert np.array_equal(got[k], a), k
    assert np.array_equal(got["img"], img)
    assert got["masses"] == {1: 1.0, 2: 1.0}


def test_data_file_reader_orders_types_and_shifts_the_box():
    """Atoms listed B first with shuffled ids, box [-2, 2): the reader returns
    A then B by id, positions relative to the lower bound, wrapped, and image
    counts for the wrap."""
    text = """LAMMPS data file written by hand

4 atoms
2 atom types

-2.0 2.0 xlo xhi
-2.0 2.0 ylo yhi
-2.0 2.0 zlo zhi

Masses

1 1.0
2 1.0

Atoms # atomic

7 2 1.5 -1.5 0.0
3 1 -2.0 0.25 1.999
9 2 2.5 0.0 0.0
1 1 0.0 0.0 -0.5

Velocities

9 0.3 0.0 0.0
1 0.1 0.2 0.3
7 -1.0 0.0 1.0
3 0.0 0.0 0.0
"""
    got = LIO.read_data(io.StringIO(text))
    assert got["n_a"] == 2 and got["L"] == 4.0
    assert got["ids"].tolist() == [1, 3, 7, 9]
    assert got["x"].tolist() == [2.0, 0.0, 3.5, 0.5]  # 2.5 lies past xhi: wrapped once
    assert got["y"].tolist() == [2.0, 2.25, 0.5, 2.0]
    assert got["img"][0].tolist() == [0, 0, 0, 1]
    assert got["vx"].tolist() == [0.1, 0.0, -1.0, 0.3]


def test_data_file_errors():
    base = "t\n\n1 atoms\n2 atom types\n\n0 1 xlo xhi\n0 1 ylo yhi\n0 2 zlo zhi\n\nAtoms\n\n1 1 0 0 0\n"
    with pytest.raises(ValueError):
        LIO.read_data(io.StringIO(base))  # not cubic
    bad_type = base.replace("0 2 zlo", "0 1 zlo").replace("1 1 0 0 0", "1 3 0 0 0")
    with pytest.raises(ValueError):
        LIO.read_data(io.StringIO(bad_type))
    with pytest.raises(ValueError):
        LIO.read_data(io.StringIO("t\n\n2 atoms\n"))


def test_dump_round_trip_with_unwrapped_columns():
    L, na, (x, y, z), v, img = _config(n=120)
    buf = io.StringIO()
    LIO.write_dump(buf, 0, x, y, z, na, L, *v)
    LIO.write_dump(buf, 50, x, y, z, na, L, *v, img=img, unwrapped=True)
    frames = LIO.read_dump(io.StringIO(buf.getvalue()))
    assert [f["step"] for f in frames] == [0, 50]
    f0, f1 = frames
    assert np.array_equal(f0["id"], np.arange(1, x.size + 1))
    assert np.array_equal(f0["type"], np.where(np.arange(x.size) < na, 1, 2))
    assert np.array_equal(f0["x"], x) and np.array_equal(f0["vz"], v[2])
    assert "xu" not in f0 and np.array_equal(f1["xu"], x + img[0] * L)
    assert np.array_equal(f1["zu"], z + img[2] * L)
    assert np.allclose(f1["box"], [[0, L]] * 3)


def test_lammps_rdf_table_matches_the_oracle_and_the_paper_normalisation():
    L, na, (x, y, z), _, _ = _config(n=600)
    n = x.size
    rcut, nbins = 2.5, 25
    h = O.rdf_hist(x, y, z, na, L, rcut / nbins, nbins)
    t = A.lammps_rdf(h, n, na, L, rcut)
    ref = O.lammps_rdf_table(h, n, na, L, rcut, nbins)
    assert t.shape == (nbins, 8)
    assert np.allclose(t, ref, rtol=1e-13, atol=0.0)
    # g columns are the paper's g (Sec. VI.A.1) on the same bins: AA, BB, AB
    _, g = A.rdf(h, n, na, L, rcut / nbins)
    assert np.allclose(t[:, 2], g[0], rtol=1e-13) and np.allclose(t[:, 4], g[2], rtol=1e-13)
    assert np.allclose(t[:, 6], g[1], rtol=1e-13)
    assert t[0, 1] == pytest.approx(0.05) and t[-1, 0] == nbins


def test_write_lammps_rdf_layout():
    t = np.zeros((3, 8))
    t[:, 0] = [1, 2, 3]
    t[:, 1] = [0.5, 1.5, 2.5]
    buf = io.StringIO()
    A.write_lammps_rdf(buf, [(200, t), (400, t)])
    lines = buf.getvalue().splitlines()
    assert lines[0].startswith("#") and lines[2].startswith("# Row")
    assert lines[3] == "200 3" and lines[4].split()[:2] == ["1", "0.5"]
    assert lines[7] == "400 3" and len(lines) == 11
