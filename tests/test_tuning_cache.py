"""Host logic of the tiling cache (no GPU): keys, hits, misses, persistence."""
import json

import paper_2406_15236_amd as mpc
from paper_2406_15236_amd import tuning


class FakeSim:
    """Stands in for a handle: records the calls the cache makes."""

    def __init__(self, boxes, form="fp64"):
        self.params = [mpc.make_params(b, form) for b in boxes]
        self.calls = []
        self.tiling = {"tile_cells": 0, "grid": 512, "yblock": 8, "order": 0, "ntiles": 99}

    def autotune(self, trial_steps):
        self.calls.append(("autotune", trial_steps))
        self.tiling.update(tile_cells=24, grid=4096, yblock=16, order=1)

    def get_tiling(self):
        return dict(self.tiling)

    def set_tiling(self, tile_cells, grid, yblock, order):
        self.calls.append(("set_tiling", tile_cells, grid, yblock, order))


def box(L, density=10.0, **kw):
    return dict(L=L, density=density, **kw)


def test_miss_then_hit(tmp_path):
    path = str(tmp_path / "cache.json")
    s1 = FakeSim([box((256, 256, 256))])
    t, hit = tuning.autotune_cached(s1, 3, path=path, device="gfx950/256cu")
    assert not hit and s1.calls == [("autotune", 3)]
    assert t == {"tile_cells": 24, "grid": 4096, "yblock": 16, "order": 1}
    s2 = FakeSim([box((256, 256, 256))])
    t2, hit2 = tuning.autotune_cached(s2, 3, path=path, device="gfx950/256cu")
    assert hit2 and t2 == t and s2.calls == [("set_tiling", 24, 4096, 16, 1)]
    data = json.load(open(path))
    assert len(data) == 1


def test_keys_separate_device_form_flags_and_shape():
    dev = "gfx950/256cu"
    k = tuning.cache_key(dev, FakeSim([box((64, 64, 64))]).params)
    assert k != tuning.cache_key("gfx942/304cu", FakeSim([box((64, 64, 64))]).params)
    assert k != tuning.cache_key(dev, FakeSim([box((64, 64, 64))], form="split").params)
    assert k != tuning.cache_key(dev, FakeSim([box((64, 64, 64), mbs=True)]).params)
    assert k != tuning.cache_key(dev, FakeSim([box((64, 64, 32))]).params)
    assert k != tuning.cache_key(dev, FakeSim([box((64, 64, 64), density=20.0)]).params)
    # large ensembles: box count, particle total and density rounded to powers of two
    many = [box((16 + i, 20, 24)) for i in range(10)]
    many2 = [box((17 + i, 20, 24)) for i in range(10)]
    assert (tuning.cache_key(dev, FakeSim(many).params)
            == tuning.cache_key(dev, FakeSim(many2).params))
    assert (tuning.cache_key(dev, FakeSim(many).params)
            != tuning.cache_key(dev, FakeSim(many[:9]).params))


def test_corrupt_file_is_a_miss(tmp_path):
    path = tmp_path / "cache.json"
    path.write_text("{not json")
    s = FakeSim([box((32, 32, 32))])
    _, hit = tuning.autotune_cached(s, 2, path=str(path), device="d")
    assert not hit and json.load(open(path))  # rewritten with the new entry
