"""Model pack (.npz) -> oracle ROMModel.  The pack format is plain arrays:
grid (nx, ny, nu, ly), split (nsx, nsy), activation, n_sub, C, and per subdomain i and
part p in {om, ga}: p{i}_W1 [w, n], p{i}_b1 [w], p{i}_W2 [N, 3, b] band values,
p{i}_xref [N], p{i}_bs = (b, s); hr{i} = sampled global node ids (ascending)."""
from __future__ import annotations

import numpy as np

from .autoencoder import Decoder
from .burgers import Grid
from .rom import ROMModel


def load_pack(pack, use_hr: bool = True) -> ROMModel:
    if isinstance(pack, str):
        pack = dict(np.load(pack, allow_pickle=False))
    g = Grid(int(pack["nx"]), int(pack["ny"]), float(pack["nu"]), float(pack["ly"]))
    n = int(pack["n_sub"])
    act = int(pack["act"])
    dec = {}
    for part in ("om", "ga"):
        dec[part] = []
        for i in range(n):
            b, s = (int(v) for v in pack[f"{part}{i}_bs"])
            dec[part].append(Decoder(np.asarray(pack[f"{part}{i}_W1"], np.float64), np.asarray(pack[f"{part}{i}_b1"], np.float64),
                                     np.asarray(pack[f"{part}{i}_W2"], np.float64), np.asarray(pack[f"{part}{i}_xref"], np.float64),
                                     b, s, act))
    hr = [np.asarray(pack[f"hr{i}"], np.int64) for i in range(n)] if use_hr else None
    return ROMModel(g, int(pack["nsx"]), int(pack["nsy"]), dec["om"], dec["ga"], hr, np.asarray(pack["C"], np.float64))
