"""Train one band-masked autoencoder on the GPU (BF16 matrix cores, FP32 master weights).

Procedure (Section 7.3): per-component min-max normalisation of the training snapshots to
[-1, 1] (a component whose range is below 1e-14 max(1, |midpoint|) keeps scale 1), 10% of the
snapshots held out, minibatches in a seeded random order every epoch, Adam at learning rate
1e-3, the rate divided by 10 after 50 epochs without a new best held-out loss, training stopped
after 300 such epochs, the weights of the best held-out loss kept.  The raw-space loss weights
each component by its normalisation scale (eq. autoencoder_AbsMSE_loss).  Every minibatch
step (forward, loss, back-propagation, Adam) runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

import seeded_inputs as si
from paper_2305_15163_amd import ddrom as dr


@dataclass
class AEResult:
    packed: np.ndarray         # best parameters, packed as the trainer's layout
    mid: np.ndarray            # normalisation midpoint per component
    scale: np.ndarray          # normalisation half-range per component
    epochs: int
    best_test: float
    history: list = field(default_factory=list)


def normalise(X: np.ndarray):
    hi, lo = X.max(axis=0), X.min(axis=0)
    mid = 0.5 * (hi + lo)
    sc = 0.5 * (hi - lo)
    sc = np.where(hi - lo < 1e-14 * np.maximum(1.0, np.abs(mid)), 1.0, sc)
    return mid, sc


def glorot_init(N: int, n: int, b: int, s: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights (masked layers: mean nonzeros per row / column as fans), zero
    biases, packed."""
    cols, valid = dr.band_slots(N, b, s)
    nnz = int(valid.sum())
    w = N * s
    seeds = si.spawn_seeds(seed, 6)
    W1e = si.glorot_uniform(nnz / w, nnz / N, (nnz,), si.rng(seeds[0]))
    W2e = si.glorot_uniform(w, n, (n, w), si.rng(seeds[2]))
    W1d = si.glorot_uniform(n, w, (w, n), si.rng(seeds[3]))
    W2d = si.glorot_uniform(nnz / N, nnz / w, (nnz,), si.rng(seeds[5]))
    return dr.ae_pack(N, n, b, s, W1e, np.zeros(w), W2e, W1d, np.zeros(w), W2d)


def train_ae(X: np.ndarray, n: int, b: int, s: int, activation: int, seed: int, epochs: int, batch: int = 32,
             lr: float = 1e-3, test_frac: float = 0.1, plateau_patience: int = 50, stop_patience: int = 300,
             init: np.ndarray | None = None, precision: int = 0, verbose: bool = False, tag: str = "") -> AEResult:
    """X: raw snapshots [n_snap][N].  `init` (packed) replaces the seeded Glorot draw;
    precision 0: BF16 operands, 1: split-BF16 (three products per tile)."""
    g = si.rng(seed)
    n_snap, N = X.shape
    perm = g.permutation(n_snap)
    n_test = max(1, int(round(test_frac * n_snap))) if n_snap > 1 else 0
    test_idx, train_idx = perm[:n_test], perm[n_test:]
    mid, sc = normalise(X[train_idx])
    Xn = torch.as_tensor(np.ascontiguousarray((X - mid) / sc, dtype=np.float32), device="cuda")
    scale = torch.as_tensor(np.ascontiguousarray(sc, dtype=np.float32), device="cuda")
    init_seed = int(g.integers(0, 2 ** 62))
    packed = init if init is not None else glorot_init(N, n, b, s, init_seed)
    tr = dr.AETrainer(N, n, b, s, activation, batch, packed, precision)

    # losses stay on the device until the end of each pass: one synchronisation per epoch
    def pass_loss(order_h, update, lr_):
        od = torch.as_tensor(np.asarray(order_h, dtype=np.int32), device="cuda")
        parts, sizes = [], []
        for k in range(0, len(order_h), batch):
            rows = od[k:k + batch]
            lt, _ = tr.step(Xn, rows, scale, lr=lr_, update=update, loss=True)
            parts.append(lt)
            sizes.append(int(rows.shape[0]))
        w = torch.as_tensor(np.asarray(sizes, dtype=np.float64), device="cuda")
        return float((torch.cat(parts).double() * w).sum().item()) / max(1, len(order_h))

    def eval_loss(idx):
        return pass_loss(idx, False, 0.0)

    best, best_p, since_best, since_plateau, plateau_best = np.inf, None, 0, 0, np.inf
    hist = []
    ep = 0
    cur_lr = lr
    for ep in range(1, epochs + 1):
        order = g.permutation(train_idx)
        tr_loss = pass_loss(order, True, cur_lr)
        te_loss = eval_loss(test_idx) if n_test else tr_loss
        hist.append((tr_loss, te_loss))
        if te_loss < plateau_best:
            plateau_best, since_plateau = te_loss, 0
        else:
            since_plateau += 1
            if since_plateau > plateau_patience:
                cur_lr *= 0.1
                since_plateau = 0
                plateau_best = te_loss
        if te_loss < best:
            best, since_best = te_loss, 0
            best_p = tr.params()          # a device copy
        else:
            since_best += 1
            if since_best > stop_patience:
                break
        if verbose and ep % 50 == 0:
            print(f"  {tag} epoch {ep}: train {tr_loss:.3e} test {te_loss:.3e} lr {cur_lr:.1e}", flush=True)
    return AEResult((best_p if best_p is not None else tr.params()).cpu().numpy(), mid, sc, ep, best, hist)
