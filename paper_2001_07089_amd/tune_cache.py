"""Persistent cache of the list parameters and step-kernel variant chosen by
``md_autotune``.

Probing every candidate skin, cell grid, block size and window setting costs
a few thousand steps, so the choice is stored in a JSON file and reused by
later runs of the same workload class on the same device.  The key is built from the device name,
the precision mode and coarse buckets of what the choice depends on: total
particle count (power of two), replica count (power of two), number density
(0.05) and mean temperature (0.25).  A hit applies the stored skin and grid
with ``md_set_list_params`` and the stored kernel variant with
``md_set_force_kernel`` (entries written before the variant was tuned carry
no variant and leave the kernel as it is); a miss runs ``md_autotune`` and
records its result.  Writes go to a temporary file that replaces the cache atomically.
"""
import json
import math
import os

from . import md

PRECISION_NAMES = {md.PREC_FP64: "fp64", md.PREC_MIXED: "mixed", md.PREC_MIXED_FIXED: "mixed_fixed"}


def default_path() -> str:
    env = os.environ.get("KAMD_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "kamd", "autotune.json")


def workload_key(device: str, precision: int, reps, dim: int = 3) -> str:
    """Cache key of a replica set (ctypes Replica array or objects with n, box,
    temperature attributes).  The density is N / L^dim; planar systems (dim 2)
    carry a "d2" part, so that they never share a key with a 3-D one."""
    reps = list(reps)
    dim = 2 if int(dim) == 2 else 3
    n_total = sum(int(r.n) for r in reps)
    rho = sum(r.n / r.box ** dim for r in reps) / len(reps)
    temp = sum(r.temperature for r in reps) / len(reps)
    parts = [
        device,
        PRECISION_NAMES.get(int(precision), str(precision)),
        f"n2^{int(math.floor(math.log2(max(n_total, 1))))}",
        f"r2^{int(math.floor(math.log2(len(reps))))}",
        f"rho{round(rho / 0.05) * 0.05:.2f}",
        f"T{round(temp / 0.25) * 0.25:.2f}",
    ]
    if dim == 2:
        parts.append("d2")
    return "|".join(parts)


def load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def store(path: str, key: str, entry: dict) -> None:
    data = load(path)
    data[key] = entry
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_name(torch_module=None) -> str:
    """The GPU as the picks depend on it: its architecture (with target
    features) and compute-unit count.  The marketing name is left out: the
    runtime reports it differently in different environments (a generic name,
    or none under some profilers)."""
    import torch
    t = torch_module or torch
    p = t.cuda.get_device_properties(t.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch}:{p.multi_processor_count}CU"


def tune(system, probe_steps: int = 100, path: str = None, device: str = None, refresh: bool = False) -> dict:
    """List parameters for ``system`` (an ``md.System``): from the cache when the
    key is present (and ``refresh`` is false), else from ``md_autotune``.
    Returns {"skin", "cell_div", "ms_per_step", "windows", "wg_size",
    "cached", "key"} (windows and wg_size None for an entry without them)."""
    path = path or default_path()
    device = device or device_name(getattr(system, "torch", None))
    key = workload_key(device, system.cfg.precision, system.reps, system.cfg.dim)
    hit = None if refresh else load(path).get(key)
    if hit and "skin" in hit and "cell_div" in hit:
        system.set_list_params(float(hit["skin"]), int(hit["cell_div"]))
        win, wg = hit.get("windows"), hit.get("wg_size")
        if win is not None and wg is not None:
            system.set_force_kernel(int(win), int(wg))
        return {"skin": float(hit["skin"]), "cell_div": int(hit["cell_div"]),
                "ms_per_step": hit.get("ms_per_step"), "windows": win, "wg_size": wg, "cached": True, "key": key}
    res = system.autotune(probe_steps)
    store(path, key, {"skin": res["skin"], "cell_div": res["cell_div"], "ms_per_step": res["ms_per_step"],
                      "windows": res["windows"], "wg_size": res["wg_size"], "probe_steps": int(probe_steps)})
    return dict(res, cached=False, key=key)
