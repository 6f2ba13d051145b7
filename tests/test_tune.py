"""Host logic of the batched form's autotuner: the coordinate descent finds
the minimum of separable and coupled costs, times each point once, and the
JSON cache round-trips by size class."""
import itertools

import pytest

from paper_2312_06538_amd import tune as T


def _brute(cost, grid):
    pts = [dict(zip(grid, v)) for v in itertools.product(*grid.values())]
    return min(pts, key=cost)


def test_descent_finds_separable_minimum():
    target = {"B": 8, "levels": 6, "hit_block": 128}
    cost = lambda p: sum((T.GRID[k].index(p[k]) - T.GRID[k].index(target[k])) ** 2 for k in p)
    best, c, seen = T.coordinate_descent(cost)
    assert best == target and c == 0
    assert len(seen) < 4 * 5 * 3          # fewer points than the whole grid
    # one axis per block finds it too
    best, c, _ = T.coordinate_descent(cost, grid=dict(T.GRID))
    assert best == target


def test_descent_handles_coupled_cost():
    # optimum of levels depends on B: deeper hierarchies for small bundles;
    # the default blocks search (B, levels) jointly
    def cost(p):
        want_levels = {4: 7, 8: 6, 16: 5, 32: 4}[p["B"]]
        return abs(p["levels"] - want_levels) + 0.1 * abs(p["B"] - 8) + (0 if p["hit_block"] == 64 else 0.5)
    best, c, _ = T.coordinate_descent(cost)
    assert c == pytest.approx(cost(_brute(cost, T.GRID)))


def test_each_point_timed_once():
    calls = []

    def cost(p):
        calls.append(T.point_key(p))
        return p["B"] + p["levels"]
    T.coordinate_descent(cost)
    assert len(calls) == len(set(calls))


def test_start_off_grid_is_rejected():
    with pytest.raises(ValueError):
        T.coordinate_descent(lambda p: 0, start={"B": 12, "levels": 5, "hit_block": 256})


def test_size_class_and_cache_roundtrip(tmp_path):
    k1 = T.size_class(64, 12_000_000, 2_400_000)
    k2 = T.size_class(64, 16_000_000, 3_000_000)
    assert k1 == k2 == "frames=64,slots=2^24,tris=2^22"
    assert T.size_class(64, 17_000_000, 3_000_000) != k1
    path = str(tmp_path / "sub" / "tune.json")
    c = T.TuneCache(path)
    assert c.get(k1) is None
    c.put(k1, {"B": 16, "levels": 5, "hit_block": 128}, 12.5)
    c2 = T.TuneCache(path)
    assert c2.get(k1) == {"B": 16, "levels": 5, "hit_block": 128}
