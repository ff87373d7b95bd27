"""Tile-size autotuner of the association kernel.

The association work item is one ordered keyframe pair times a tile of the
source frame's valid-pixel list (a multiple of 256 pixels, run by 256 threads
with 1, 2, 4 or 8 pixels each).  The best tile depends on the resolution and
the number of keyframes (how many items a launch has to fill 256 CUs with).
This module times whole optimisations on the GPU for each candidate tile and
keeps a JSON table keyed by "<width>x<height>/<node bucket>".  The table
shipped beside this module is handed to the library when it is loaded
(pg_set_tile_table): a graph whose Config.tile_pixels is 0 takes its class's
tile, and every graph of a batch keeps its own.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, Iterable, Optional, Sequence

TILES = (256, 512, 768, 1024, 1536, 2048)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")
BATCH_KEY = "batch"   # table key of a whole batched schedule (one tile for every window)
NODE_BUCKETS = ((2, 7), (8, 11), (12, 15), (16, 32))


def bucket_key(width: int, height: int, n_frames: int) -> str:
    for lo, hi in NODE_BUCKETS:
        if lo <= n_frames <= hi:
            return f"{width}x{height}/{lo}-{hi}"
    return f"{width}x{height}/other"


def time_optimize(make_graphs: Callable[[int], Sequence], tile: int, steps: int = 10, warmup: int = 3) -> float:
    """Median wall time (ms) of one optimize (or batched optimize) of the
    graphs make_graphs(tile) returns, poses reset before every call."""
    import torch

    from .posegraph import optimize_batch
    pgs, inits = make_graphs(tile)
    times = []
    for k in range(warmup + steps):
        for pg, P in zip(pgs, inits):
            pg.set_poses(P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if len(pgs) == 1:
            pgs[0].optimize()
        else:
            optimize_batch(pgs)
        torch.cuda.synchronize()
        if k >= warmup:
            times.append(1000.0 * (time.perf_counter() - t0))
    for pg in pgs:
        pg.close()
    times.sort()
    return times[len(times) // 2]


def tune(classes: Dict[str, Callable[[int], Sequence]], tiles: Iterable[int] = TILES, steps: int = 10,
         log: Optional[Callable[[str], None]] = print) -> Dict[str, dict]:
    """For each class (key -> graph factory taking the tile size), time every
    tile and keep the fastest.  Returns {key: {"tile": t, "ms": {tile: ms}}}."""
    table = {}
    for key, make in classes.items():
        ms = {}
        for t in tiles:
            ms[t] = time_optimize(make, t, steps=steps)
            if log:
                log(f"autotune {key}: tile {t} -> {ms[t]:.3f} ms")
        best = min(ms, key=ms.get)
        table[key] = {"tile": int(best), "ms": {str(k): round(v, 4) for k, v in ms.items()}}
    return table


def save(table: Dict[str, dict], path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path: str) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(table: Dict[str, dict], width: int, height: int, n_frames: int, default: int = 0) -> int:
    """Tuned tile for a window (0 = the library's own choice)."""
    e = table.get(bucket_key(width, height, n_frames))
    return int(e["tile"]) if e else default


def parse_key(key: str):
    """(width, height, min_frames, max_frames) of a class key, or None (the
    batch key and unbounded buckets)."""
    try:
        res, bucket = key.split("/")
        w, h = (int(x) for x in res.split("x"))
        lo, hi = (int(x) for x in bucket.split("-"))
    except ValueError:
        return None
    return w, h, lo, hi


def table_entries(table: Dict[str, dict]):
    """The library's records {width, height, min_frames, max_frames, tile}
    of every class entry of a table."""
    out = []
    for key in sorted(table):
        k = parse_key(key)
        if k is not None:
            out.append((*k, int(table[key]["tile"])))
    return out


def apply(table: Dict[str, dict], lib=None) -> int:
    """Hand a table's class entries to the library; returns their count."""
    import ctypes as C

    from . import _lib
    lib = lib or _lib.load()
    ent = table_entries(table)
    arr = (C.c_int * (5 * max(len(ent), 1)))(*[v for e in ent for v in e])
    rc = lib.pg_set_tile_table(arr, len(ent))
    if rc != 0:
        raise RuntimeError(f"pg_set_tile_table: {lib.pose_graph_last_error(None).decode()}")
    return len(ent)


def pixels_per_thread(tile: int) -> int:
    """Pixels per thread of the kernel that runs a tile (as the library picks)."""
    p = -(-tile // 256)
    for q in (1, 2, 4, 8):
        if q >= p:
            return q
    return 8


def tune_classes(graphs: Sequence, make: Callable[[object, int], Sequence], tiles: Iterable[int] = TILES,
                 steps: int = 10, log: Optional[Callable[[str], None]] = print) -> Dict[str, dict]:
    """One entry per class of `graphs` (their resolution and node bucket):
    the class's largest window is optimised alone with every tile
    (make(window, tile) -> (graphs, start poses)) and the fastest kept."""
    rep = {}
    for g in graphs:
        key = bucket_key(g.width, g.height, g.n_frames)
        if key not in rep or g.n_frames > rep[key].n_frames:
            rep[key] = g
    return tune({key: (lambda t, w=w: make(w, t)) for key, w in sorted(rep.items())}, tiles, steps, log)
