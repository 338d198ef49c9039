"""The JSON cache of launch choices (host logic only): the first call times
the variants and writes the file, a later call reads it and hands the
stored choices to the library instead of timing again; entries of other
devices or model widths are kept apart."""
import json

from paper_2212_11296_amd import api, tuning
from workloads import CONFIGS, MULTI_LATTICE


def test_cache_round_trip(tmp_path, monkeypatch):
    calls = {"tune": 0, "set": []}

    def fake_autotune(cfg, params, spins, mode=api.DEDUP, ws=None,
                      budget=None):
        calls["tune"] += 1
        return [1, 2, 4]

    def fake_set(cfg, choices):
        calls["set"].append(list(choices))

    monkeypatch.setattr(api, "autotune", fake_autotune)
    monkeypatch.setattr(api, "set_tuning", fake_set)
    path = str(tmp_path / "t.json")
    cfg = api.make_config(CONFIGS["large"])
    ch, cached = tuning.autotune_cached(cfg, None, None, path,
                                        device_name="devA")
    assert (ch, cached, calls["tune"]) == ([1, 2, 4], False, 1)
    data = json.load(open(path))
    assert data == {"devA|d=128|seg=128": {"qkv_mb": 1, "mlp_mb": 2,
                                           "vq_mb": 4}}
    ch, cached = tuning.autotune_cached(cfg, None, None, path,
                                        device_name="devA")
    assert (ch, cached, calls["tune"]) == ([1, 2, 4], True, 1)
    assert calls["set"] == [[1, 2, 4]]
    # another device, another width: timed and stored beside the first
    tuning.autotune_cached(cfg, None, None, path, device_name="devB")
    tuning.autotune_cached(api.make_config(CONFIGS["grad"]), None, None,
                           path, device_name="devA")
    assert calls["tune"] == 3
    assert sorted(json.load(open(path))) == [
        "devA|d=128|seg=128", "devA|d=256|seg=256", "devB|d=128|seg=128"]
    # the multi-lattice models share one width: one entry serves them all
    keys = {tuning.cache_key(api.make_config(mc), "devA")
            for mc in MULTI_LATTICE}
    assert keys == {"devA|d=128|seg=128"}


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert tuning.load(str(p)) == {}
    assert tuning.load(str(tmp_path / "missing.json")) == {}
