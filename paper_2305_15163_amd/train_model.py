"""Train every subdomain autoencoder of a model on the GPU and write the model pack.

Input: a skeleton pack (grid, split, hyper-reduction nodes, C and the training recipe, without
decoders) and the FOM state snapshot matrix [n_snap][N_x] with the subdomains' interior and
interface index lists, as written by the offline pipeline's skeleton mode.  For each subdomain
the interior and the interface autoencoder are trained by `train_ae.train_ae` (Section 7.3:
per-component normalisation, 10% held out, Adam with plateau decay and early stopping, BF16
matrix-core products with FP32 masters), in several processes that share the GPU.  Each
trained decoder is exported as the online solve reads it (eq. autoencoder_architecture b/d):
the de-normalisation folded into W2 and x_ref, and the latent origin moved to the mean encoded
training snapshot (b1 <- b1 + W1 m, which leaves the trial manifold unchanged).

Usage:  python -m paper_2305_15163_amd.train_model <stem> --out models/<name>.npz [--procs 8]
        (<stem>_skel.npz, <stem>_X.npy, <stem>_X_dd.npz)
        In parts: --only om0,ga0,... --subset-to <stem2> (write those autoencoders' columns), then
        train <stem2> --only ... --out part.npz on each part, then --merge part*.npz --out pack.npz.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ACT_SIGMOID, ACT_SWISH, ACT_IDENTITY = 0, 1, 2


def _act(z: np.ndarray, act: int) -> np.ndarray:
    if act == ACT_IDENTITY:
        return z
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg if act == ACT_SIGMOID else z * sg


def unpack_weights(packed, N: int, n: int, b: int, s: int) -> dict:
    """The trainer's packed FP32 parameters as dense-index weights: the encoder's masked layer
    as (column c, row r, value) triplets, the two dense layers and biases, the decoder's band
    slots [N][3][b] (zero where a slot's column lies outside [0, w))."""
    from paper_2305_15163_amd import ddrom as dr
    w1e, b1e, W2e, W1d, b1d, w2d = dr.ae_unpack(packed, N, n, b, s)
    cols, valid = dr.band_slots(N, b, s)
    flat_valid = np.flatnonzero(valid.ravel())
    rows = np.broadcast_to(np.arange(N)[:, None, None], cols.shape).ravel()[flat_valid]
    c = cols.ravel()[flat_valid]
    order = np.lexsort((rows, c))          # the encoder's entries are listed by (c, r)
    vals = np.zeros(cols.shape)
    vals[valid] = w2d
    return dict(enc_c=c[order], enc_r=rows[order], enc_v=w1e, b1e=b1e, W2e=W2e, W1d=W1d, b1d=b1d, W2d=vals)


def encode(wts: dict, Xn: np.ndarray, w: int, act: int) -> np.ndarray:
    """Latents of normalised snapshots Xn [m][N] (FP64 on the host)."""
    import scipy.sparse as sp
    E1 = sp.csr_matrix((wts["enc_v"], (wts["enc_c"], wts["enc_r"])), shape=(w, Xn.shape[1]))
    return _act((E1 @ Xn.T).T + wts["b1e"], act) @ wts["W2e"].T


def decode_full(wts: dict, xh: np.ndarray, N: int, b: int, s: int, act: int) -> np.ndarray:
    """Normalised reconstructions [m][N] of latents xh [m][n]."""
    a = _act(xh @ wts["W1d"].T + wts["b1d"], act)              # [m][w]
    out = np.zeros((xh.shape[0], N))
    w = a.shape[1]
    for k in range(3):
        for t in range(b):
            c = np.arange(N) * s + (k - 1) * b * s + t
            ok = (c >= 0) & (c < w)
            out[:, ok] += a[:, c[ok]] * wts["W2d"][ok, k, t]
    return out


def export_decoder(wts: dict, mid: np.ndarray, sc: np.ndarray, center: np.ndarray, b: int, s: int) -> dict:
    return dict(W1=wts["W1d"].copy(), b1=wts["b1d"] + wts["W1d"] @ center, W2=wts["W2d"] * sc[:, None, None],
                xref=mid.copy(), bs=np.array([b, s]))


def raw_decoder(wts: dict, mid: np.ndarray, sc: np.ndarray, center: np.ndarray, b: int, s: int) -> dict:
    """What export_decoder is formed from, in half the bytes: the trained decoder weights are FP32
    values, so they are stored in FP32 (losslessly) beside the FP64 normalisation and centre."""
    return dict(W1=wts["W1d"].astype(np.float32), b1=wts["b1d"].astype(np.float32),
                W2=wts["W2d"].astype(np.float32), sc=sc.copy(), mid=mid.copy(), center=center.copy(),
                bs=np.array([b, s]))


def decoder_from_raw(r: dict) -> dict:
    """export_decoder of the weights raw_decoder stored (the same values, formed the same way)."""
    b, s = (int(v) for v in r["bs"])
    wts = dict(W1d=np.asarray(r["W1"], dtype=np.float64), b1d=np.asarray(r["b1"], dtype=np.float64),
               W2d=np.asarray(r["W2"], dtype=np.float64))
    return export_decoder(wts, np.asarray(r["mid"]), np.asarray(r["sc"]), np.asarray(r["center"]), b, s)


def _job(args):
    """One autoencoder, in its own process: train on the GPU, export, and measure the relative
    reconstruction error on the held-out snapshots (host FP64 evaluation of the trained
    weights)."""
    stem, xpath, tag, i, n, b, s, act, seed, epochs, batch, precision, raw = args
    import torch  # noqa: F401  (initialises the device in this process)
    from paper_2305_15163_amd.train_ae import train_ae
    import seeded_inputs as si
    idx = np.load(stem + "_X_dd.npz")[f"{tag}{i}"]
    Xall = np.load(xpath, mmap_mode="r")                      # FP64, or FP32 to move less data
    X = np.ascontiguousarray(Xall[:, idx], dtype=np.float64)
    t0 = time.time()
    res = train_ae(X, n, b, s, act, seed, epochs, batch=batch, precision=precision, verbose=True, tag=f"{tag}{i}")
    dt = time.time() - t0
    N = X.shape[1]
    wts = unpack_weights(res.packed, N, n, b, s)
    g = si.rng(seed)                      # the held-out split train_ae drew
    perm = g.permutation(X.shape[0])
    n_test = max(1, int(round(0.1 * X.shape[0]))) if X.shape[0] > 1 else 0
    test_idx, train_idx = perm[:n_test], perm[n_test:]
    Xn_tr = (X[train_idx] - res.mid) / res.scale
    center = encode(wts, Xn_tr, N * s, act).mean(axis=0)
    dec = (raw_decoder if raw else export_decoder)(wts, res.mid, res.scale, center, b, s)
    Xt = X[test_idx] if n_test else X[train_idx]
    rec = decode_full(wts, encode(wts, (Xt - res.mid) / res.scale, N * s, act), N, b, s, act) * res.scale + res.mid
    rel = np.linalg.norm(rec - Xt, axis=1) / np.maximum(1e-300, np.linalg.norm(Xt, axis=1))
    rep = dict(ae=f"{tag}{i}", N=N, latent=n, epochs=res.epochs, best_test_loss=res.best_test, seconds=dt,
               steps=res.epochs * -(-len(train_idx) // batch), rel_rec_err_mean=float(rel.mean()),
               rel_rec_err_max=float(rel.max()))
    return tag, i, dec, rep


def train_model(stem: str, procs: int = 8, epochs: int | None = None, precision: int = 0, verbose: bool = True,
                snapshots: str | None = None, only=None, raw: bool = False):
    """snapshots: the state snapshot matrix (default <stem>_X.npy).  only: the autoencoders to
    train (tags such as "om0", "ga3"; default: every autoencoder the index-list file names); the
    pack then holds only their decoders (see merge).  raw: the pack holds only the decoders, as
    raw_decoder stores them (<tag>_raw_<key>), for merge to finish with the skeleton."""
    skel = dict(np.load(stem + "_skel.npz", allow_pickle=False))
    xpath = snapshots or stem + "_X.npy"
    n_sub = int(skel["n_sub"])
    b, s = (int(v) for v in skel["train_bs"])
    act = int(skel["act"])
    ep = int(skel["train_epochs"]) if epochs is None else int(epochs)
    batch = int(skel["train_batch"])
    import seeded_inputs as si
    seeds = si.spawn_seeds(int(skel["train_seed"]), 2 * n_sub)
    jobs = []
    idx = np.load(stem + "_X_dd.npz")
    for i in range(n_sub):
        jobs.append((stem, xpath, "om", i, int(skel["train_n_om"][i]), b, s, act, seeds[2 * i], ep, batch,
                     precision, raw))
        jobs.append((stem, xpath, "ga", i, int(skel["train_n_ga"][i]), b, s, act, seeds[2 * i + 1], ep, batch,
                     precision, raw))
    if not only:     # a subset written by subset_data holds only its autoencoders' index lists
        only = [t for t in idx.files if t[:2] in ("om", "ga") and t[2:].isdigit()]
    jobs = [j for j in jobs if f"{j[2]}{j[3]}" in set(only)]
    jobs.sort(key=lambda j: -len(idx[f"{j[2]}{j[3]}"]))     # largest first
    t0 = time.time()
    if procs > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(min(procs, len(jobs))) as pool:
            out = []
            for r in pool.imap_unordered(_job, jobs):
                out.append(r)
                if verbose:
                    print("[train_model]", json.dumps(r[3]), flush=True)
    else:
        out = []
        for j in jobs:
            out.append(_job(j))
            if verbose:
                print("[train_model]", json.dumps(out[-1][3]), flush=True)
    pack = {} if raw else {k: v for k, v in skel.items() if not k.startswith("train_")}
    reports = []
    for tag, i, dec, rep in out:
        for key, v in dec.items():
            pack[f"{tag}{i}_raw_{key}" if raw else f"{tag}{i}_{key}"] = v
        reports.append(rep)
    reports.sort(key=lambda r: r["ae"])
    return pack, reports, time.time() - t0


def merge(paths, out, skeleton: str | None = None):
    """One pack from packs that each hold some subdomains' trained decoders (the rest equal).
    Parts written with raw=True hold only decoders: their exported form is formed here
    (decoder_from_raw) and the rest of the pack comes from the skeleton <skeleton>_skel.npz."""
    pack = {}
    if skeleton:
        skel = np.load(skeleton + "_skel.npz", allow_pickle=False)
        pack.update({k: skel[k] for k in skel.files if not k.startswith("train_")})
    for p in paths:
        part = np.load(p, allow_pickle=False)
        raws = {}
        for k in part.files:
            if "_raw_" in k:
                tag, key = k.split("_raw_")
                raws.setdefault(tag, {})[key] = part[k]
            else:
                pack.setdefault(k, part[k])
        if raws and not skeleton:
            raise ValueError(f"{p} holds raw decoders: give the skeleton to merge them")
        for tag, r in raws.items():
            for key, v in decoder_from_raw(r).items():
                pack.setdefault(f"{tag}_{key}", v)
    np.savez(out, **pack)
    return pack


def grid_rows(mus: np.ndarray, every: int) -> np.ndarray:
    """Rows of a snapshot matrix on a tensor parameter grid (mus [n_snap][2]) whose two grid
    indices are both multiples of `every`: a coarser tensor grid over the same box."""
    ia = np.searchsorted(np.unique(mus[:, 0]), mus[:, 0])
    il = np.searchsorted(np.unique(mus[:, 1]), mus[:, 1])
    return np.flatnonzero((ia % every == 0) & (il % every == 0))


def subset_data(stem: str, tags, out_stem: str, snapshots: str | None = None, every: int = 1):
    """The snapshot columns the autoencoders `tags` read (FP32) with their index lists renumbered,
    and the skeleton, under out_stem: training data for `train_model --only` that is smaller than
    the whole matrix (for moving it to another machine).  every > 1 keeps only the snapshots of
    the coarser parameter grid (grid_rows; the parameters come from the matrix's _dd file)."""
    import shutil
    idx = np.load(stem + "_X_dd.npz")
    xpath = snapshots or stem + "_X.npy"
    X = np.load(xpath, mmap_mode="r")
    rows = slice(None)
    if every > 1:
        rows = grid_rows(np.load(os.path.splitext(xpath)[0] + "_dd.npz")["mus"], every)
    cols = np.unique(np.concatenate([idx[t] for t in tags]))
    pos = np.full(X.shape[1], -1, dtype=np.int64)
    pos[cols] = np.arange(len(cols))
    Xs = np.asarray(X[rows], dtype=np.float32) if every > 1 else X
    np.save(out_stem + "_X.npy", np.asarray(Xs[:, cols], dtype=np.float32))
    np.savez(out_stem + "_X_dd.npz", **{t: pos[idx[t]] for t in tags})
    shutil.copy(stem + "_skel.npz", out_stem + "_skel.npz")
    return len(cols)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--merge", nargs="+", default=None, help="packs to merge into --out (no training)")
    ap.add_argument("--subset-to", default=None, help="with --only: write the columns those autoencoders read "
                                                      "(and the skeleton) under this stem; no training")
    ap.add_argument("--only", default=None, help="comma-separated autoencoders to train (e.g. om0,ga0)")
    ap.add_argument("stem", nargs="?")
    ap.add_argument("--out", default=None)
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=None, help="override the recipe's epoch count")
    ap.add_argument("--precision", type=int, default=0, help="0: BF16 operands, 1: split-BF16")
    ap.add_argument("--snapshots", default=None, help="state snapshot matrix (default <stem>_X.npy)")
    ap.add_argument("--raw", action="store_true", help="write only the decoders, in FP32 where they are "
                                                        "FP32 values (about half the bytes); --merge with "
                                                        "--skeleton then forms the pack")
    ap.add_argument("--skeleton", default=None, help="with --merge: the skeleton stem of raw parts")
    ap.add_argument("--every", type=int, default=1, help="with --subset-to: keep every k-th parameter of "
                                                         "the snapshot grid in both directions")
    a = ap.parse_args(argv)
    if a.merge:
        merge(a.merge, a.out, a.skeleton)
        print(f"[train_model] merged {len(a.merge)} packs into {a.out}", flush=True)
        return 0
    if a.subset_to:
        n = subset_data(a.stem, a.only.split(","), a.subset_to, a.snapshots, a.every)
        print(f"[train_model] wrote {n} columns under {a.subset_to}", flush=True)
        return 0
    pack, reports, dt = train_model(a.stem, a.procs, a.epochs, a.precision, snapshots=a.snapshots,
                                    only=a.only.split(",") if a.only else None, raw=a.raw)
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    np.savez(a.out, **pack)
    with open(os.path.splitext(a.out)[0] + "_train.json", "w") as f:
        json.dump(dict(seconds=dt, autoencoders=reports), f, indent=1)
    print(f"[train_model] wrote {a.out} ({dt:.0f}s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
