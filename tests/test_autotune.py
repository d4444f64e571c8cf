"""Host logic of the per-class launch tuner: the cache key depends on the batch's (Nx, Nz)
histogram (not on tank order), the precision and the device; a missing or corrupt cache reads as
empty; the search visits the classes heaviest first, keeps each class's fastest candidate and
stores the choice."""
import sys
import types

from paper_2406_00991_amd import autotune


def test_cache_key_and_load(tmp_path):
    k1 = autotune._key([64, 128, 64], [9, 17, 9], "mixed", "dev")
    k2 = autotune._key([128, 64, 64], [17, 9, 9], "mixed", "dev")
    assert k1 == k2
    assert k1 != autotune._key([64, 128, 64], [9, 17, 9], "fp64", "dev")
    assert k1 != autotune._key([64, 128, 64], [9, 17, 9], "mixed", "other")
    assert k1 != autotune._key([64, 128], [9, 17], "mixed", "dev")
    bad = tmp_path / "c.json"
    bad.write_text("{not json")
    assert autotune._load(str(bad)) == {}
    assert autotune._load(str(tmp_path / "missing.json")) == {}


def test_candidates_per_class():
    assert autotune.candidates(33, "mixed") == [(512, 2), (256, 2), (128, 2)]
    assert autotune.candidates(17, "mixed")[0] == (256, 1)
    assert autotune.candidates(17, "fp64") == [(512, 2), (256, 2), (128, 2)]


def test_search_keeps_fastest_candidate_per_class(tmp_path, monkeypatch):
    # a synthetic cost: one term per class, each class with a known best choice
    best = {33: (512, 2), 9: (256, 1)}
    seen = []

    def fake_time(nx, nz, L, h, eo, en, b, precision, opts, rtol=1e-10, reps=2):
        ct, cr = list(opts.class_threads), list(opts.class_resident)
        seen.append((ct, cr))
        cost = 0.0
        for rows, (t, r) in best.items():
            c = autotune.pmgw.CLASS_ROWS.index(rows)
            cost += 10.0 if (ct[c], cr[c]) == (t, r) else 20.0 + ct[c] / 100.0
        return cost

    monkeypatch.setattr(autotune, "time_batch", fake_time)
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(get_device_name=lambda: "dev"))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    cache = str(tmp_path / "tune.json")
    choice, log = autotune.tune([512, 64], [33, 9], [1.0, 1.0], None, None, None, None,
                                precision="mixed", cache=cache)
    assert choice["class_threads"][4] == 512 and choice["class_resident"][4] == 2
    assert choice["class_threads"][2] == 256 and choice["class_resident"][2] == 1
    assert [r[0] for r in log] == [33] * 3 + [9] * 4          # heaviest class first
    again, log2 = autotune.tune([64, 512], [9, 33], [1.0, 1.0], None, None, None, None,
                                precision="mixed", cache=cache)
    assert again == choice and log2 is None                   # read back from the cache
