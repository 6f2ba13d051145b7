"""Autotuner of the batched form: bundle size B, hierarchy depth and the
workgroup size of the final tests, chosen by timing the captured batch.

The search is block coordinate descent over the grid B x levels x
hit_block (the merge factor stays at its value): the bundle size and the
depth trade off against each other (smaller bundles want deeper trees), so
they form one block searched jointly; each block in turn takes every value
combination with the other parameters held, the best point so far is kept,
and rounds repeat until a round changes nothing.  Every point is timed at
most once.  Results are cached in a JSON file keyed by the batch's size
class (frame count, and the powers of two bounding its total ray slots and
triangles), so batches of the same class reuse them.
"""
import itertools
import json
import math
import os

GRID = {"B": (4, 8, 16, 32), "levels": (3, 4, 5, 6, 7), "hit_block": (64, 128, 256)}
START = {"B": 16, "levels": 5, "hit_block": 256}
BLOCKS = (("B", "levels"), ("hit_block",))


def point_key(p):
    return ",".join(f"{k}={p[k]}" for k in sorted(p))


def coordinate_descent(cost, start=None, grid=None, blocks=None, max_rounds=4):
    """Minimise cost(point) over the product grid by block coordinate
    descent (blocks: tuples of axis names searched jointly; default one
    block per axis when a grid is given, BLOCKS for the default grid).
    Returns (best point, its cost, {point_key: cost} of every timed point)."""
    if grid is None:
        grid = GRID
        blocks = blocks or BLOCKS
    blocks = blocks or tuple((k,) for k in grid)
    best = dict(start or START)
    for k, axis in grid.items():
        if best[k] not in axis:
            raise ValueError(f"start {k}={best[k]} is not on the grid")
    seen = {point_key(best): cost(best)}
    best_c = seen[point_key(best)]
    for _ in range(max_rounds):
        moved = False
        for names in blocks:
            for vals in itertools.product(*(grid[k] for k in names)):
                cand = dict(best, **dict(zip(names, vals)))
                key = point_key(cand)
                if key not in seen:
                    seen[key] = cost(cand)
                if seen[key] < best_c:
                    best, best_c, moved = cand, seen[key], True
        if not moved:
            break
    return best, best_c, seen


def size_class(n_frames, total_slots, total_tris):
    """Cache key: frame count and the powers of two at or above the totals."""
    lr = max(0, math.ceil(math.log2(max(total_slots, 1))))
    lt = max(0, math.ceil(math.log2(max(total_tris, 1))))
    return f"frames={n_frames},slots=2^{lr},tris=2^{lt}"


def default_cache_path():
    return os.environ.get("CRSH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "crsh_tune.json"))


class TuneCache:
    """{size class: {"params": point, "ms": time}} in a JSON file."""

    def __init__(self, path=None):
        self.path = path or default_cache_path()
        self.data = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, key):
        e = self.data.get(key)
        return dict(e["params"]) if e else None

    def put(self, key, params, ms):
        self.data[key] = {"params": dict(params), "ms": float(ms)}
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def time_graph_ms(db, stream, reps=3):
    """Median time (ms) of `reps` replays of the batch's captured graph,
    after one eager run that sizes the pair arrays."""
    import torch
    db.run_with_retry()
    g = db.graph(stream)
    try:
        g.launch()                       # warm-up
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.launch()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        m, st = db.read_meta(stream)
        if st != 0:                      # a replay overflowed: not a valid point
            return float("inf")
        return sorted(ts)[len(ts) // 2]
    finally:
        g.close()


def tune_batch(db, stream, cache=None, reps=3, log=None):
    """Tune (B, levels, hit_block) for a DeviceBatch; the batch is left
    reshaped to the best point.  Uses / fills the cache when given."""
    key = size_class(db.n_frames, db.cap, db.m)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            db.reshape(hit["B"], db.F, hit["levels"], hit["hit_block"])
            return hit, None, {}

    def cost(p):
        db.reshape(p["B"], db.F, p["levels"], p["hit_block"])
        ms = time_graph_ms(db, stream, reps)
        if log:
            log(f"[tune] {point_key(p)}: {ms:.3f} ms")
        return ms

    best, ms, seen = coordinate_descent(cost)
    db.reshape(best["B"], db.F, best["levels"], best["hit_block"])
    if cache is not None:
        cache.put(key, best, ms)
    return best, ms, seen
