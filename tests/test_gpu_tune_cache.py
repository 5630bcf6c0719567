"""The shipped autotuner picks apply on this GPU: the cache key of the
device the tests run on is the one the shipped file was written for."""
import os

import pytest

from paper_2001_07089_amd import md, tune_cache

pytestmark = pytest.mark.gpu


def test_shipped_picks_hit_on_this_device():
    data = tune_cache.load(os.path.join(os.path.dirname(md.__file__), "tuned", "autotune.json"))
    dev = tune_cache.device_name()
    print("device key", dev, flush=True)
    assert any(k.startswith(dev + "|") for k in data), (dev, list(data))
