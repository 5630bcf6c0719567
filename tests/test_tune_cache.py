"""Host logic of the autotuner cache: keys, hit/miss behaviour, atomic JSON
storage.  The two library calls are replaced by recording fakes, so this runs
without a GPU."""
import json
import os
import types

import pytest

from paper_2001_07089_amd import md, tune_cache
from paper_2001_07089_amd import workload as W


def _system(reps, precision="mixed_fixed"):
    """Stands in for md.System: its autotune / set_list_params call the
    library functions, which the fixture replaces."""
    cfg = md.make_config(precision)
    s = types.SimpleNamespace(ctx="CTX", cfg=cfg, reps=md.make_replicas(reps))
    s.autotune = lambda probe_steps=100: md.md_autotune(s.ctx, probe_steps)
    s.set_list_params = lambda skin, cell_div=1: md.md_set_list_params(s.ctx, skin, cell_div)
    s.set_force_kernel = lambda windows, wg_size=0: md.md_set_force_kernel(s.ctx, windows, wg_size)
    return s


@pytest.fixture
def fakes(monkeypatch):
    calls = {"tune": 0, "set": [], "kernel": []}

    def fake_tune(ctx, probe_steps=100):
        calls["tune"] += 1
        return {"skin": 0.4, "cell_div": 1, "ms_per_step": 0.43, "windows": 1, "wg_size": 128}

    def fake_set(ctx, skin, cell_div):
        calls["set"].append((skin, cell_div))

    def fake_kernel(ctx, windows, wg_size=0):
        calls["kernel"].append((windows, wg_size))

    monkeypatch.setattr(md, "md_autotune", fake_tune)
    monkeypatch.setattr(md, "md_set_list_params", fake_set)
    monkeypatch.setattr(md, "md_set_force_kernel", fake_kernel)
    return calls


def test_miss_then_hit(tmp_path, fakes):
    r = W.ka_large().replicas[0]
    s = _system([(r.n, r.n_a, r.box, r.temperature, r.seed)])
    path = str(tmp_path / "c" / "tune.json")
    a = tune_cache.tune(s, 50, path=path, device="MI355X:gfx950")
    assert not a["cached"] and fakes["tune"] == 1 and fakes["set"] == []
    b = tune_cache.tune(s, 50, path=path, device="MI355X:gfx950")
    assert b["cached"] and fakes["tune"] == 1 and fakes["set"] == [(0.4, 1)]
    assert fakes["kernel"] == [(1, 128)]
    assert (b["skin"], b["cell_div"], b["windows"], b["wg_size"]) == \
        (a["skin"], a["cell_div"], a["windows"], a["wg_size"])
    data = json.load(open(path))
    assert list(data) == [a["key"]] and data[a["key"]]["probe_steps"] == 50
    c = tune_cache.tune(s, 50, path=path, device="MI355X:gfx950", refresh=True)
    assert not c["cached"] and fakes["tune"] == 2


def test_key_separates_device_precision_and_workload():
    r = W.ka_large().replicas[0]
    one = md.make_replicas([(r.n, r.n_a, r.box, r.temperature, r.seed)])
    k = tune_cache.workload_key("dev", md.PREC_MIXED_FIXED, one)
    assert k != tune_cache.workload_key("other", md.PREC_MIXED_FIXED, one)
    assert k != tune_cache.workload_key("dev", md.PREC_FP64, one)
    small = W.ka_small().replicas[0]
    assert k != tune_cache.workload_key("dev", md.PREC_MIXED_FIXED,
                                        md.make_replicas([(small.n, small.n_a, small.box, 0.45, 1)]))
    batch = W.ka_batch_small()
    kb = tune_cache.workload_key("dev", md.PREC_MIXED, md.make_replicas(batch.replicas))
    assert "r2^8" in kb and "rho1.20" in kb
    # a different seed (same class) maps to the same key
    assert k == tune_cache.workload_key("dev", md.PREC_MIXED_FIXED,
                                        md.make_replicas([(r.n, r.n_a, r.box, r.temperature, r.seed + 7)]))
    # a planar system: its own key, with the density N / L^2
    p = W.ka_planar(1 << 20, 0.4).replicas[0]
    flat = md.make_replicas([(p.n, p.n_a, p.box, p.temperature, p.seed)])
    kp = tune_cache.workload_key("dev", md.PREC_MIXED_FIXED, flat, dim=2)
    assert kp.endswith("|d2") and "rho1.20" in kp
    assert kp != tune_cache.workload_key("dev", md.PREC_MIXED_FIXED, flat)
    assert "d2" not in k


def test_corrupt_cache_is_a_miss(tmp_path, fakes):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    r = W.ka_small().replicas[0]
    s = _system([(r.n, r.n_a, r.box, r.temperature, r.seed)], "fp64")
    out = tune_cache.tune(s, 10, path=str(path), device="d")
    assert not out["cached"] and fakes["tune"] == 1
    assert out["key"] in json.load(open(path))


def test_device_name_is_arch_and_compute_units():
    """The key leaves out the marketing name, which the runtime reports
    differently in different environments (empty under some profilers)."""
    props = types.SimpleNamespace(name="", gcnArchName="gfx950:sramecc+:xnack-", multi_processor_count=256)
    fake = types.SimpleNamespace(cuda=types.SimpleNamespace(current_device=lambda: 0,
                                                            get_device_properties=lambda i: props))
    assert tune_cache.device_name(fake) == "gfx950:sramecc+:xnack-:256CU"
    props.name = "AMD Radeon Graphics"
    assert tune_cache.device_name(fake) == "gfx950:sramecc+:xnack-:256CU"


def test_shipped_picks_are_well_formed():
    data = tune_cache.load(os.path.join(os.path.dirname(md.__file__), "tuned", "autotune.json"))
    assert data
    for key, e in data.items():
        assert key.count("|") == 5 or (key.count("|") == 6 and key.endswith("|d2"))
        assert 0.2 <= e["skin"] <= 0.5 and e["cell_div"] in (1, 2)
        assert e["windows"] in (0, 1) and e["wg_size"] in (64, 128, 256)
