"""Persisted table of work-item shapes, one entry per model bucket.

A bucket is (grid, subdomain split, per-subdomain latent sizes, per-subdomain hyper-reduction
node counts, batch size, precision): models in one bucket have identical kernel work, so a
shape measured for one serves the others.  Missing entries are measured with the library's
ddrom_autotune (coordinate search over the decoder, residual and constraint work-item shapes,
median of timed batched solves) and written back.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from paper_2305_15163_amd import ddrom as dr


def bucket(pack: dict, B: int, precision: int) -> str:
    n = int(pack["n_sub"])
    lat = [(int(np.asarray(pack[f"om{i}_W1"]).shape[1]), int(np.asarray(pack[f"ga{i}_W1"]).shape[1])) for i in range(n)]
    hr = [int(np.asarray(pack[f"hr{i}"]).shape[0]) for i in range(n)]
    digest = hashlib.sha1(json.dumps([lat, hr]).encode()).hexdigest()[:12]
    return f"{int(pack['nx'])}x{int(pack['ny'])}/{int(pack['nsx'])}x{int(pack['nsy'])}/{digest}/B{int(B)}/p{int(precision)}"


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(path: str, table: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tiles_for(pack: dict, mu, o: dr.Opts, path: str | None = None, reps: int = 5, verbose: bool = False):
    """Shape for this pack and batch: from the table at `path` if present, else measured (and
    stored when `path` is given)."""
    key = bucket(pack, len(mu), o.precision)
    table = load(path) if path else {}
    if key in table:
        return tuple(table[key]["tile"])
    tile, rows = dr.autotune_tiles(pack, mu, o, reps=reps)
    if verbose:
        for r in rows:
            print(f"  [autotune {key}] tile {r[:3]} {r[3]:.3f} ms", flush=True)
        print(f"  [autotune {key}] chose {tile}", flush=True)
    if path:
        table = load(path)
        table[key] = dict(tile=list(tile), tried=[list(r) for r in rows])
        save(path, table)
    return tile
