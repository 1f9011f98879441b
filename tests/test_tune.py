"""The autotuner's cache, on the host: the Python reader's fallback to the
built-in shapes on a missing or corrupt file, and the library's own loader
(syn_autotune_load): strict parsing, all-or-nothing replacement, stale entries
(another build) skipped, exact-shape lookup, and the precedence of an explicit
lane count over the table."""
import json

import pytest

from paper_2410_01136_amd import binding as sm
from paper_2410_01136_amd import tune


@pytest.fixture(autouse=True)
def clean_table():
    sm.syn_autotune_clear()
    yield
    sm.syn_autotune_clear()
    for k in range(3):
        for kind in range(5):
            sm.set_lanes_per_ray(k, kind, 0)


def key(dev="*", bid=None, k=0, f=1, p=786432, n=512, q=3, grid=False):
    bid = bid or sm.syn_build_id().decode()
    return f"{dev}|{bid}|k{k}|f{f}|p{p}|n{n}|q{q}" + ("|g" if grid else "")


def lookup(k=0, f=1, p=786432, n=512, q=3):
    lanes, mode = sm._i32(), sm._i32()
    hit = sm.syn_autotune_lookup(k, f, p, n, q, sm.ctypes.byref(lanes), sm.ctypes.byref(mode))
    return (lanes.value, mode.value) if hit else None


def test_python_cache_reader_falls_back_on_missing_or_corrupt_files(tmp_path):
    assert tune.load_cache(str(tmp_path / "absent.json")) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert tune.load_cache(str(bad)) == {}
    bad.write_text(json.dumps([1, 2, 3]))
    assert tune.load_cache(str(bad)) == {}
    mixed = tmp_path / "mixed.json"
    mixed.write_text(json.dumps({"a": 16, "b": 5, "c": [4, 3], "d": [4, 1], "e": "x", "f": True,
                                 "x|k0|y": 8, "x|k1|y": [8, 2], "x|k2|y": 8}))
    # 8 lanes per sightline: forward and reverse entries only, not batch ones
    assert tune.load_cache(str(mixed)) == {"a": 16, "c": [4, 3], "x|k0|y": 8, "x|k1|y": [8, 2]}


def test_library_loads_entries_of_this_build_and_looks_up_exact_shapes(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({
        key(grid=True): [4, 2],
        key(k=1, f=0, p=49152, n=768, q=1): 16,
        key(bid="0000000000000000", k=2, f=0, p=100, n=10, q=1): 64,  # another build: stale
        key(dev="Some Other GPU", k=0, f=0, p=3072, n=256, q=1): 1,
    }, indent=1))
    assert tune.load(str(p)) == 3
    assert lookup() == (4, 2)
    assert lookup(k=1, f=0, p=49152, n=768, q=1) == (16, 0)
    assert lookup(k=2, f=0, p=100, n=10, q=1) is None      # stale entry skipped
    assert lookup(p=786431) is None and lookup(n=511) is None and lookup(q=2) is None
    assert lookup(k=0, f=0, p=3072, n=256, q=1) is None    # not this device


@pytest.mark.parametrize("text,msg", [
    (None, "cannot open"),
    ("", "expected '{'"),
    ("{", "expected"),
    ('{"%s": 16,}', "expected"),
    ('{"%s": 5}', "lane count"),
    ('{"%s": [16, 1]}', "grid read mode"),
    ('{"%s": 16.5}', "expected"),
    ('{"a|b|k0": 16}', "malformed key"),
    ('{"%s": 16} trailing', "trailing"),
])
def test_library_loader_rejects_bad_files_and_keeps_its_table(tmp_path, text, msg):
    good = tmp_path / "good.json"
    good.write_text(json.dumps({key(): 16}))
    assert tune.load(str(good)) == 1
    p = tmp_path / "bad.json"
    if text is not None:
        p.write_text(text.replace("%s", key()) if "%s" in text else text)
    with pytest.raises(sm.SynError) as e:
        tune.load(str(p))
    assert e.value.status == sm.SYN_EINVAL and msg in str(e.value)
    assert sm.syn_autotune_entries() == 1 and lookup() == (16, 0)


def test_eight_lanes_are_accepted_for_marches_and_refused_for_batch_entries(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({key(k=1, f=1, p=49152, n=768, q=1): 8}))
    assert tune.load(str(p)) == 1
    assert lookup(k=1, f=1, p=49152, n=768, q=1) == (8, 0)
    p.write_text(json.dumps({key(k=2, f=0, p=100, n=10, q=1): 8}))
    with pytest.raises(sm.SynError) as e:
        tune.load(str(p))
    assert e.value.status == sm.SYN_EINVAL and "batch" in str(e.value)
    assert lookup(k=1, f=1, p=49152, n=768, q=1) == (8, 0)  # table unchanged


def test_grid_flag_and_value_shape_must_agree(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({key(grid=False): [4, 3]}))
    with pytest.raises(sm.SynError):
        tune.load(str(p))
    p.write_text(json.dumps({key(grid=True): 4}))
    with pytest.raises(sm.SynError):
        tune.load(str(p))


def test_explicit_lane_count_beats_the_table(tmp_path):
    # without a device the forward cannot launch, so the precedence is read
    # through the public getters: the table answers for its exact shape, the
    # process-wide setter overrides every shape of its kernel and field kind
    p = tmp_path / "t.json"
    p.write_text(json.dumps({key(k=0, f=0, p=3072, n=256, q=1): 1}))
    tune.load(str(p))
    assert lookup(k=0, f=0, p=3072, n=256, q=1) == (1, 0)
    sm.set_lanes_per_ray(0, 0, 16)
    assert sm.get_lanes_per_ray(0, 0, 3072) == 16
