"""FOM reference states for the error measure of eq. relative_error (Section 7), written once by
the oracle and read by the benchmark as data.

Each named set is a list of held-out parameters (a, lambda) drawn as the benchmark draws them
(seeded_inputs.heldout_mu(count, seed), its first `take` entries; optionally the paper's test
point mu* of Section 7.1 first) and the monolithic FOM Newton states on the given grid.

Usage:
  python -m oracle.fom_reference --grid 240 240 --set batch:1:512:64 --set proposal:5:2048:64 \
      --out models/cfg1_fomref.npz [--workers 8]
  python -m oracle.fom_reference --grid 480 24 --mu-star --set heldout:7:64:64 --lam-range 5 25 \
      --out models/paper_fomref.npz
  python -m oracle.fom_reference --grid 480 480 --set uneven:2:1024:8:2/3 --out models/cfg2c_fomref.npz

A fifth field k/m keeps only the draws that seeded_inputs.model_assignment(count, m, seed) gives
to model k (the uneven batch's split of its parameters over m models), then the first `take`.

The file holds, per set name s: s_mu [n][2], s_x [n][N_x] (the FP64 Newton states rounded to FP32:
their relative rounding, 6e-8, is far below the errors measured against them), and
fom_s_per_solve (mean wall time of one Newton solve on one core of the machine that wrote it).
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import seeded_inputs as si
from .burgers import BurgersFOM, Grid, solve_fom

MU_STAR = (7692.5384, 21.9230)      # the paper's test point (Section 7.1)


def _job(args):
    nx, ny, mu = args
    t0 = time.perf_counter()
    r = solve_fom(BurgersFOM(Grid(nx, ny)), mu)
    return r.x, bool(r.converged), time.perf_counter() - t0


def states(nx: int, ny: int, mus: np.ndarray, workers: int = 8):
    jobs = [(nx, ny, tuple(float(v) for v in m)) for m in mus]
    if workers > 1:
        with ProcessPoolExecutor(workers) as ex:
            out = list(ex.map(_job, jobs, chunksize=1))
    else:
        out = [_job(j) for j in jobs]
    if not all(o[1] for o in out):
        raise RuntimeError("FOM Newton did not converge for some reference parameter")
    return np.stack([o[0] for o in out]), float(np.mean([o[2] for o in out]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, nargs=2, required=True)
    ap.add_argument("--set", action="append", default=[], help="name:seed:count:take")
    ap.add_argument("--mu-star", action="store_true", help="also the set 'star' holding mu* alone")
    ap.add_argument("--lam-range", type=float, nargs=2, default=None, help="lambda range of the held-out draws")
    ap.add_argument("--out", required=True)
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args(argv)
    nx, ny = a.grid
    out, times = {"grid": np.array([nx, ny])}, []
    sets = []
    if a.mu_star:
        sets.append(("star", np.array([MU_STAR], dtype=np.float64)))
    for spec in a.set:
        name, seed, count, take, *part = spec.split(":")
        lr = tuple(a.lam_range) if a.lam_range else si.LAM_RANGE
        mus = si.heldout_mu(int(count), int(seed), lam_range=lr)
        if part:
            k, m = (int(v) for v in part[0].split("/"))
            mus = mus[si.model_assignment(int(count), m, int(seed)) == k]
        sets.append((name, mus[:int(take)]))
    for name, mus in sets:
        t0 = time.time()
        X, ts = states(nx, ny, mus, a.workers)
        out[f"{name}_mu"] = mus
        out[f"{name}_x"] = X.astype(np.float32)     # FP64 solves; FP32 storage keeps the file small
        times.append(ts)
        print(f"[fom_reference] {name}: {len(mus)} states in {time.time() - t0:.0f}s", flush=True)
    out["fom_s_per_solve"] = np.float64(np.mean(times))
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    np.savez(a.out, **out)
    print("wrote", a.out, flush=True)
    return 0


if __name__ == "__main__":
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    sys.exit(main())
