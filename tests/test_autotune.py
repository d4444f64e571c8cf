"""Host logic of the workgroup-size tuner: the cache key depends on the batch's (Nx, Nz)
histogram (not on tank order), the precision and the device; a missing or corrupt cache reads as
empty."""
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
