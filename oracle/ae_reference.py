"""FP64 CPU-trained reference autoencoder for GPU training runs (Section 7.3 recipe).

Trains one subdomain autoencoder with the oracle (FP64, hand-written gradients, Adam) on the
columns of a FOM snapshot matrix that belong to it, and writes what a GPU run of the same
architecture, seed, held-out split, initial weights and minibatch order is compared with: the
held-out loss history and the relative reconstruction error ||x - g(h(x))|| / ||x|| of the
held-out snapshots in raw (de-normalised) space.

Usage:
  python -m oracle.ae_reference --stem models/snap/cfg3_X --part om --sd 5 --n 8 --b 9 --s 2 \
      --seed <seed> --epochs 60 --batch 64 --out models/cfg3_ae_ref_om5.json
(<stem>.npy: snapshots [n_snap][N_x]; <stem>_dd.npz: the subdomains' index lists.)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import seeded_inputs as si
from .autoencoder import ACT_SIGMOID, MaskedAE, act, train


def held_out_error(ae: MaskedAE, p, nm, X: np.ndarray, seed: int, test_frac: float = 0.1):
    """Relative reconstruction error of the held-out snapshots (the split train() drew)."""
    g = si.rng(seed)
    perm = g.permutation(X.shape[0])
    n_test = max(1, int(round(test_frac * X.shape[0]))) if X.shape[0] > 1 else 0
    Xt = X[perm[:n_test]]
    Xn = (Xt - nm.m) / nm.s
    xh = ae.encode(p, Xn)
    ad, _ = act(xh @ p.W1d.T + p.b1d, ae.act)
    Y = (ae._dec_mat(p) @ ad.T).T * nm.s + nm.m
    rel = np.linalg.norm(Y - Xt, axis=1) / np.maximum(1e-300, np.linalg.norm(Xt, axis=1))
    return rel


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stem", required=True)
    ap.add_argument("--part", choices=("om", "ga"), required=True)
    ap.add_argument("--sd", type=int, required=True)
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--b", type=int, required=True)
    ap.add_argument("--s", type=int, required=True)
    ap.add_argument("--act", type=int, default=ACT_SIGMOID)
    ap.add_argument("--seed", type=int, required=True)
    ap.add_argument("--epochs", type=int, required=True)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    idx = np.load(a.stem + "_dd.npz")[f"{a.part}{a.sd}"]
    X = np.ascontiguousarray(np.load(a.stem + ".npy", mmap_mode="r")[:, idx])
    ae = MaskedAE(X.shape[1], a.n, a.b, a.s, a.act)
    t0 = time.time()
    p, nm, rep = train(ae, X, a.seed, a.epochs, batch=a.batch, verbose=True)
    dt = time.time() - t0
    rel = held_out_error(ae, p, nm, X, a.seed)
    out = dict(part=a.part, sd=a.sd, N=int(X.shape[1]), n=a.n, b=a.b, s=a.s, act=a.act, seed=a.seed,
               epochs=int(rep.epochs), batch=a.batch, best_test_loss=float(rep.test_loss),
               test_loss_history=[float(h[1]) for h in rep.history], rel_rec_err_mean=float(rel.mean()),
               rel_rec_err_max=float(rel.max()), seconds=dt, precision="fp64")
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "test_loss_history"}), flush=True)
    return 0


if __name__ == "__main__":
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    sys.exit(main())
