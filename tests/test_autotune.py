"""Host logic of the autotuner: the coordinate search and the cache."""

import itertools

from paper_1709_03802_amd import autotune as AT


def test_coordinate_search_finds_separable_minimum():
    space = {"a": [0, 1, 2, 3], "b": [5, 6, 7], "c": [0, 1]}
    target = {"a": 2, "b": 7, "c": 1}

    def cost(s):
        return sum((s[k] - target[k]) ** 2 for k in s) + 1.0

    best, c, log = AT.coordinate_search(space, cost)
    assert best == target and c == 1.0
    # never more evaluations than one sweep per round plus the start
    assert len(log) <= 1 + 2 * sum(len(v) - 1 for v in space.values())


def test_coordinate_search_never_worse_than_start():
    space = {"x": [0, 1, 2], "y": [0, 1, 2]}
    table = {(x, y): ((x * 7 + y * 3) % 5) + 0.5 * (x == y) for x, y in itertools.product(range(3), range(3))}
    start = {"x": 1, "y": 2}
    best, c, log = AT.coordinate_search(space, lambda s: table[(s["x"], s["y"])], start=start)
    assert c <= table[(1, 2)]
    assert c == min(v for _, v in log)


def test_space_drops_tiles_at_or_above_the_wavelength_count():
    assert AT.space_for(4)["lambda_tile"] == [0, 1]
    assert AT.space_for(32)["lambda_tile"] == [0, 1, 4, 8, 16]
    assert AT.space_for(1)["lambda_tile"] == [0]


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert AT.load_cache(p) == {}
    k = AT.cache_key("dev", 4096, 8, 8, "scatter")
    AT.save_cache({k: {"setting": {"lambda_tile": 0, "block_waves": 2}, "ms": 1.5}}, p)
    got = AT.load_cache(p)
    assert got[k]["setting"]["block_waves"] == 2
    assert k != AT.cache_key("dev", 4096, 8, 4, "scatter")
