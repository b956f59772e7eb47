"""Host-side checks of the autotuner: its candidate space, the conservative
reference candidate, the cache file, and the plan fields it sets (validated
by the library without a GPU)."""
import ctypes
import json

import pytest

from paper_1201_2501_amd import autotune, sfft


def test_default_space_exact_respects_kernel_limits():
    sp = autotune.default_space(1 << 22, 256, sfft.SFFT_MODE_EXACT)
    assert sp["bins"]["B"] == [512, 1024, 2048, 4096]
    assert set(sp["launch"]["hash_threads"]) == {256, 512, 1024}
    small = autotune.default_space(1 << 14, 16, sfft.SFFT_MODE_EXACT)
    assert max(small["bins"]["B"]) <= (1 << 14) // 16
    gen = autotune.default_space(1 << 26, 1024, sfft.SFFT_MODE_GENERAL)
    assert gen["bins"]["B"] == [4096]


def test_reference_candidate_is_the_conservative_corner():
    sp = autotune.default_space(1 << 22, 256, sfft.SFFT_MODE_EXACT)
    ref = autotune.reference_candidate(sp, sfft.SFFT_MODE_EXACT, {"theta": 0.02})
    assert ref["B"] == 4096 and ref["delta"] == 1e-10 and ref["b_min"] == 64 and ref["patience"] == 5
    assert ref["alpha"] == 0.5
    assert ref["theta"] == 0.02 and ref["hash_threads"] == 256 and ref["chunks"] == 1


def test_every_candidate_field_is_a_plan_field_that_validates():
    lib = sfft.load()
    sp = autotune.default_space(1 << 22, 256, sfft.SFFT_MODE_EXACT)
    base = {"B": 1024, "b_min": 64, "patience": 4, "rounds": 24}
    for stage in sp.values():
        for f, values in stage.items():
            for v in values:
                cand = autotune.normalize(dict(base, **{f: v}))
                d = sfft.sfft_desc_init(1 << 22, 256, 1024)
                for name, val in cand.items():
                    setattr(d, name, val)
                assert lib.sfft_validate_params(ctypes.byref(d)) == sfft.SFFT_OK, (f, v)


def test_group0_offset_is_relative_to_the_library_default():
    # B = 1024 reaches b_min = 64 at round 4; patience 4 -> default group 0 of 9 rounds
    assert autotune.first_floor_round(1024, 64) == 4 and autotune.first_floor_round(1024, 2048) == 0
    c = autotune.normalize({"B": 1024, "b_min": 64, "patience": 4, "rounds": 24, "group0_offset": 2})
    assert c["group0"] == 11 and "group0_offset" not in c
    assert "group0" not in autotune.normalize({"B": 1024, "b_min": 64, "group0_offset": 0})


@pytest.mark.parametrize("field,value", [("hash_threads", 128), ("hash_threads", 768), ("chunks", 9),
                                         ("stop_patience", 0), ("group0", 33), ("group_step", 33),
                                         ("hash_order", 3)])
def test_launch_shape_fields_are_validated(field, value):
    lib = sfft.load()
    d = sfft.sfft_desc_init(1 << 20, 64, 512)
    setattr(d, field, value)
    assert lib.sfft_validate_params(ctypes.byref(d)) == sfft.SFFT_EINVAL


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tuned.json")
    key = autotune.cache_key(1 << 20, 64, 0, 32, 0, "test-device")
    autotune._store_cache(path, key, {"B": 512, "fields": {"b_min": 32, "hash_threads": 512}, "ms": 1.5,
                                      "rate": 21333.3, "quality": 1.0})
    hit = autotune.lookup(path, 1 << 20, 64, 0, 32, 0, "test-device")
    assert hit.from_cache and hit.B == 512 and hit.fields["hash_threads"] == 512
    assert autotune.lookup(path, 1 << 20, 64, 0, 64, 0, "test-device") is None      # other batch size
    assert autotune.lookup(path, 1 << 20, 64, 0, 32, 0, "other-device") is None
    assert json.load(open(path))[key]["ms"] == 1.5
    assert autotune.lookup(str(tmp_path / "missing.json"), 1 << 20, 64, 0, 32, 0, "test-device") is None
    # another build's entry serves when asked, marked as such
    other = autotune.lookup(path, 1 << 20, 64, 0, 32, 0, "test-device", any_build=True)
    assert other.from_cache is True
    data = json.load(open(path))
    data[key.replace("|lib=", "|lib=old")] = data.pop(key)
    json.dump(data, open(path, "w"))
    assert autotune.lookup(path, 1 << 20, 64, 0, 32, 0, "test-device") is None
    stale = autotune.lookup(path, 1 << 20, 64, 0, 32, 0, "test-device", any_build=True)
    assert stale.from_cache == "other build" and stale.B == 512
