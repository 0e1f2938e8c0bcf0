"""The autotuner on the device: it returns a valid setting no slower than the default, caches it,
and the moments under the tuned launch shape still match the oracle."""
import json

import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import tune
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_tune_and_cache(tmp_path):
    op = wl.spin_cubic_lattice(24, seed=81)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    h = kpm.Hamiltonian(op, a, b, kpm.F64)
    cache = str(tmp_path / "tune.json")
    before = kpm.get_launch()
    res = tune.tune([h], 3, wl.VEC_PHASE, keys=["march_items", "xcd_split"], steps=4, passes=1, cache=cache)
    assert kpm.get_launch() == before
    assert res["seconds_per_step"] <= res["default_seconds_per_step"]
    assert set(res["settings"]) == {"march_items", "xcd_split"}
    stored = json.load(open(cache))
    assert res["key"] in stored
    again = tune.tune([h], 3, wl.VEC_PHASE, cache=cache)
    assert again["cached"] and again["settings"] == res["settings"]
    with kpm.launch_settings(**res["settings"]):
        mu = kpm.moments(h, 64, 3, wl.VEC_PHASE, 9, 0).cpu().numpy()
    ref = gu.oracle_moments(op, a, b, 64, 3, wl.VEC_PHASE, 9, 0)
    gu.assert_fp64(mu, ref, "tuned launch shape")
    h.free()
