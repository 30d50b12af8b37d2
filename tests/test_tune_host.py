"""Host logic of the autotuner: candidates, signatures and the cache file."""
import json

from paper_2403_10647_amd import tune


def test_candidates_cover_the_space():
    c = tune.candidates()
    assert len(c) == 4 * 5 * 2
    assert tune.DEFAULTS in c
    assert all(set(k) == set(tune.KNOBS) for k in c)
    small = tune.candidates({"max_digit_bits": (9,), "sort_shape": (0, 3), "fused_expand": (0,)})
    assert small == [{"max_digit_bits": 9, "sort_shape": 0, "fused_expand": 0},
                     {"max_digit_bits": 9, "sort_shape": 3, "fused_expand": 0}]


def test_signature_groups_by_bits_and_magnitude():
    assert tune.signature(False, 25, 51_023_216) == "plain:bits25:pairs2^25"
    assert tune.signature(False, 25, 40_000_000) == tune.signature(False, 25, 51_023_216)
    assert tune.signature(True, 25, 51_023_216) != tune.signature(False, 25, 51_023_216)
    assert tune.signature(False, 22, 51_023_216) != tune.signature(False, 25, 51_023_216)
    assert tune.signature(False, 1, 0) == "plain:bits1:pairs2^0"


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    knobs = {"max_digit_bits": 10, "sort_shape": 2, "fused_expand": 0}
    c = tune.record({}, "dev", "plain:bits25:pairs2^25", knobs, 1.25, [{"knobs": knobs, "ms": 1.25}])
    tune.save_cache(path, c)
    back = tune.load_cache(path)
    assert tune.lookup(back, "dev", "plain:bits25:pairs2^25") == knobs
    assert tune.lookup(back, "other", "plain:bits25:pairs2^25") is None
    assert tune.lookup(back, "dev", "plain:bits22:pairs2^25") is None


def test_corrupt_cache_is_ignored(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert tune.load_cache(str(p)) == {}
    p.write_text(json.dumps({"dev": {"s": {"knobs": {"max_digit_bits": 9}}}}))
    assert tune.lookup(tune.load_cache(str(p)), "dev", "s") is None   # incomplete entry
