"""LAMMPS data and dump files for one replica (Sec. IV.B).

The paper's LAMMPS runs start from a data file (atom style atomic: a header
with the atom count, two atom types and the box, then the Masses, Atoms and
Velocities sections) and write dump snapshots with the columns id, type, x,
y, z, vx, vy, vz, sorted by id.  These helpers read and write those formats
so that a configuration can move between this library and LAMMPS.

Conventions.  Type 1 is A and type 2 is B.  The library's caller order holds
a replica's A particles first, then its B particles; read_data returns that
order (the file's ids sorted within each type) together with the ids.  The
box is cubic, [lo, lo + L) in every direction; positions are returned
relative to lo and wrapped into [0, L).  Image flags, when the Atoms lines
carry them, are returned as img (3 x n), so that x + img * L is unwrapped.
"""
import io
from typing import Dict, List

import numpy as np


def _open(f, mode):
    if isinstance(f, (str, bytes)) or hasattr(f, "__fspath__"):
        return open(f, mode), True
    return f, False


def write_data(f, x, y, z, n_a: int, L: float, vx=None, vy=None, vz=None, img=None,
               masses=(1.0, 1.0), title: str = "KA binary Lennard-Jones configuration"):
    """Write one replica (caller order: A then B) as a LAMMPS data file.  Ids
    are 1..n in caller order.  With img given, each Atoms line also carries
    the image flags ix iy iz."""
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    n = x.size
    fh, own = _open(f, "w")
    try:
        fh.write(f"# {title}\n\n")
        fh.write(f"{n} atoms\n2 atom types\n\n")
        for a in ("x", "y", "z"):
            fh.write(f"0 {L:.17g} {a}lo {a}hi\n")
        fh.write("\nMasses\n\n")
        fh.write(f"1 {masses[0]:.17g}\n2 {masses[1]:.17g}\n")
        fh.write("\nAtoms # atomic\n\n")
        im = None if img is None else np.asarray(img, np.int64)
        for i in range(n):
            t = 1 if i < n_a else 2
            line = f"{i + 1} {t} {x[i]:.17g} {y[i]:.17g} {z[i]:.17g}"
            if im is not None:
                line += f" {im[0][i]} {im[1][i]} {im[2][i]}"
            fh.write(line + "\n")
        if vx is not None:
            vx, vy, vz = (np.asarray(a, np.float64) for a in (vx, vy, vz))
            fh.write("\nVelocities\n\n")
            for i in range(n):
                fh.write(f"{i + 1} {vx[i]:.17g} {vy[i]:.17g} {vz[i]:.17g}\n")
    finally:
        if own:
            fh.close()


_SECTIONS = ("Masses", "Atoms", "Velocities")


def read_data(f) -> Dict[str, object]:
    """Read a LAMMPS data file with two atom types and a cubic box.  Returns
    dict(n, n_a, L, ids, x, y, z, vx, vy, vz, img, masses) in caller order (A
    then B, each by increasing id); vx.. are None without a Velocities
    section, img is None without image flags."""
    fh, own = _open(f, "r")
    try:
        lines = fh.read().splitlines()
    finally:
        if own:
            fh.close()
    n = None
    ntypes = None
    lo = {}
    hi = {}
    body: Dict[str, List[str]] = {}
    cur = None
    for raw in lines[1:]:  # the first line is the title
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        word = line.split()[0]
        if word in _SECTIONS:
            cur = word
            body[cur] = []
            continue
        if cur is None:
            tok = line.split()
            if len(tok) >= 2 and tok[1] == "atoms":
                n = int(tok[0])
            elif len(tok) >= 3 and tok[1:3] == ["atom", "types"]:
                ntypes = int(tok[0])
            elif len(tok) >= 4 and tok[2].endswith("lo") and tok[3].endswith("hi"):
                lo[tok[2][0]] = float(tok[0])
                hi[tok[2][0]] = float(tok[1])
            continue
        body[cur].append(line)
    if n is None or "Atoms" not in body:
        raise ValueError("not a LAMMPS data file: atom count or Atoms section missing")
    if ntypes not in (1, 2):
        raise ValueError(f"expected 1 or 2 atom types, found {ntypes}")
    Ls = {a: hi[a] - lo[a] for a in "xyz"} if set(lo) >= set("xyz") else None
    if Ls is None or max(Ls.values()) - min(Ls.values()) > 1e-12 * max(Ls.values()):
        raise ValueError("expected a cubic box with xlo xhi, ylo yhi, zlo zhi")
    L = Ls["x"]
    rows = [r.split() for r in body["Atoms"]]
    if len(rows) != n:
        raise ValueError(f"Atoms section holds {len(rows)} lines for {n} atoms")
    ids = np.array([int(r[0]) for r in rows], np.int64)
    typ = np.array([int(r[1]) for r in rows], np.int64)
    if not np.all((typ == 1) | (typ == 2)):
        raise ValueError("atom types must be 1 (A) or 2 (B)")
    pos = np.array([[float(v) for v in r[2:5]] for r in rows], np.float64)
    has_img = all(len(r) >= 8 for r in rows)
    im = np.array([[int(v) for v in r[5:8]] for r in rows], np.int64) if has_img else None
    order = np.lexsort((ids, typ))  # A first, by id
    out = {"n": n, "n_a": int(np.count_nonzero(typ == 1)), "L": L, "ids": ids[order]}
    shift = np.array([lo["x"], lo["y"], lo["z"]])
    p = pos[order] - shift
    k = np.floor(p / L)
    p = p - k * L
    p[p >= L] = 0.0
    out["x"], out["y"], out["z"] = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    base = np.zeros((3, n), np.int64) if im is None else im[order].T
    wrapped = k.T.astype(np.int64)
    out["img"] = (base + wrapped).astype(np.int32) if (im is not None or np.any(wrapped)) else None
    if "Velocities" in body:
        vel = {int(r.split()[0]): [float(v) for v in r.split()[1:4]] for r in body["Velocities"]}
        v = np.array([vel[int(i)] for i in out["ids"]], np.float64)
        out["vx"], out["vy"], out["vz"] = v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
    else:
        out["vx"] = out["vy"] = out["vz"] = None
    masses = {}
    for r in body.get("Masses", []):
        t = r.split()
        masses[int(t[0])] = float(t[1])
    out["masses"] = masses
    return out


def write_dump(f, step: int, x, y, z, n_a: int, L: float, vx=None, vy=None, vz=None, img=None,
               unwrapped: bool = False):
    """Append one snapshot in the LAMMPS dump custom layout, sorted by id
    (ids 1..n in caller order): columns id type x y z, then vx vy vz when
    given, then xu yu zu (x + img L) when unwrapped is set (img required)."""
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    n = x.size
    cols = ["id", "type", "x", "y", "z"]
    data = [np.arange(1, n + 1), np.where(np.arange(n) < n_a, 1, 2), x, y, z]
    if vx is not None:
        cols += ["vx", "vy", "vz"]
        data += [np.asarray(vx, np.float64), np.asarray(vy, np.float64), np.asarray(vz, np.float64)]
    if unwrapped:
        if img is None:
            raise ValueError("unwrapped coordinates need the image counters")
        im = np.asarray(img, np.float64)
        cols += ["xu", "yu", "zu"]
        data += [x + im[0] * L, y + im[1] * L, z + im[2] * L]
    fh, own = _open(f, "a")
    try:
        fh.write(f"ITEM: TIMESTEP\n{int(step)}\nITEM: NUMBER OF ATOMS\n{n}\n")
        fh.write("ITEM: BOX BOUNDS pp pp pp\n" + f"0 {L:.17g}\n" * 3)
        fh.write("ITEM: ATOMS " + " ".join(cols) + "\n")
        buf = io.StringIO()
        for i in range(n):
            buf.write(f"{int(data[0][i])} {int(data[1][i])} " +
                      " ".join(f"{c[i]:.17g}" for c in data[2:]) + "\n")
        fh.write(buf.getvalue())
    finally:
        if own:
            fh.close()


def read_dump(f) -> List[Dict[str, object]]:
    """Read every snapshot of a dump custom file: a list of dicts with step,
    n, box (3 x 2) and one array per column, rows sorted by id."""
    fh, own = _open(f, "r")
    try:
        lines = fh.read().splitlines()
    finally:
        if own:
            fh.close()
    frames = []
    i = 0
    while i < len(lines):
        if not lines[i].startswith("ITEM: TIMESTEP"):
            i += 1
            continue
        step = int(lines[i + 1].split()[0])
        if not lines[i + 2].startswith("ITEM: NUMBER OF ATOMS"):
            raise ValueError("malformed dump: atom count missing")
        n = int(lines[i + 3].split()[0])
        if not lines[i + 4].startswith("ITEM: BOX BOUNDS"):
            raise ValueError("malformed dump: box bounds missing")
        box = np.array([[float(v) for v in lines[i + 5 + k].split()[:2]] for k in range(3)])
        head = lines[i + 8]
        if not head.startswith("ITEM: ATOMS"):
            raise ValueError("malformed dump: ATOMS header missing")
        cols = head.split()[2:]
        rows = np.array([[float(v) for v in lines[i + 9 + k].split()] for k in range(n)], np.float64)
        rows = rows[np.argsort(rows[:, cols.index("id")], kind="stable")] if "id" in cols else rows
        fr = {"step": step, "n": n, "box": box}
        for k, c in enumerate(cols):
            fr[c] = rows[:, k].astype(np.int64) if c in ("id", "type") else rows[:, k]
        frames.append(fr)
        i += 9 + n
    return frames


def replica_arrays(system, replica: int = 0) -> Dict[str, object]:
    """Host copies of one replica of an md.System (caller order), ready for
    write_data / write_dump: x, y, z, vx, vy, vz, img, n_a, L."""
    a = system.numpy(("x", "y", "z", "vx", "vy", "vz"))
    img = system.images()
    sl = system.replica_slice(replica)
    r = system.reps[replica]
    out = {k: v[sl].copy() for k, v in a.items()}
    out["img"] = np.asarray(img)[:, sl].copy()
    out["n_a"] = int(r.n_a)
    out["L"] = float(r.box)
    return out
