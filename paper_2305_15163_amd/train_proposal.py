"""Train the proposal network of a model pack on the method's own solutions (GPU).

    python -m paper_2305_15163_amd.train_proposal models/cfg1.npz --out models/cfg1_mlp.npz

1. draws the training parameters (uniform over the box, seeded) and solves them with
   rom_solve_batch (FP64, relative KKT tolerance 1e-8);
2. takes the converged [xhat; lambda] as targets, standardised per component;
3. trains the network (2 -> 256 -> 256 -> n_D + n_C, SiLU) with the library's forward,
   back-propagation and Adam kernels on minibatches of 256 for the given epochs, 10% of the
   rows held out; the weights with the lowest held-out loss (checked every 25 epochs) are
   kept, since the network overfits the 3.7k training rows well before 2000 epochs;
4. writes sizes, FP32 parameters, the standardisation and the loss history to --out.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import seeded_inputs as si  # noqa: E402
from paper_2305_15163_amd import ddrom as dr  # noqa: E402


def solve_targets(model, mus: np.ndarray, batch: int = 512, max_iter: int = 60):
    ws = dr.Workspace(model, min(batch, len(mus)))
    o = dr.opts(max_iter=max_iter, tol_rel=1e-8, precision=dr.PREC_FP64)
    X, L, S = [], [], []
    for s0 in range(0, len(mus), batch):
        r = dr.rom_solve_batch(model, ws, mus[s0:s0 + batch], o)
        X.append(r["xhat"].cpu().numpy())
        L.append(r["lam"][:, :model.n_C].cpu().numpy())
        S.append(r["status"].cpu().numpy())
    return np.concatenate(X), np.concatenate(L), np.concatenate(S)


def standardise(Y: np.ndarray):
    m = Y.mean(axis=0)
    s = Y.std(axis=0)
    s = np.where(s < 1e-12, 1.0, s)
    return m, s


def train(model_pack: dict, n_train: int = 4096, seed: int = 4, epochs: int = 2000, batch: int = 256,
          hidden=(256, 256), lr: float = 1e-3, check_every: int = 25, verbose: bool = True,
          mus: np.ndarray | None = None):
    """Returns the proposal pack (dict of numpy arrays)."""
    t0 = time.perf_counter()
    model = dr.Model(model_pack)
    if mus is None:
        mus = si.heldout_mu(n_train, seed)
    X, L, S = solve_targets(model, mus)
    keep = S == 0
    mus_k, Y = mus[keep], np.concatenate([X, L], axis=1)[keep]
    n_D, n_C = model.n_D, model.n_C
    if verbose:
        print(f"[proposal] {keep.sum()} of {len(mus)} training solves converged "
              f"({time.perf_counter() - t0:.1f}s)", flush=True)
    mean, std = standardise(Y)
    Tn = ((Y - mean) / std).astype(np.float32)
    sizes = [2, *hidden, n_D + n_C]
    init = si.mlp_init(sizes, seed)
    tr = dr.ProposalTrainer(sizes, dr.pack_mlp_params(init), max_batch=batch)
    N = len(mus_k)
    train_idx, test_idx = si.train_split(N, 0.1, seed)
    mu_d = torch.as_tensor(np.ascontiguousarray(mus_k), dtype=torch.float64, device="cuda")
    T_d = torch.as_tensor(np.ascontiguousarray(Tn), device="cuda")
    hist = []
    best = (np.inf, 0, None)

    def eval_loss(idx):
        tot, cnt = 0.0, 0
        for s0 in range(0, len(idx), batch):
            rows = torch.as_tensor(idx[s0:s0 + batch], dtype=torch.int32, device="cuda")
            lt, _ = tr.step(mu_d, T_d, rows, update=False, loss=True)
            tot += float(lt.item()) * len(rows)
            cnt += len(rows)
        return tot / max(1, cnt)

    for ep in range(epochs):
        order = torch.as_tensor(train_idx[si.epoch_order(len(train_idx), seed, ep)], dtype=torch.int32, device="cuda")
        for s0 in range(0, len(order), batch):
            tr.step(mu_d, T_d, order[s0:s0 + batch], lr=lr)
        if (ep + 1) % check_every == 0 or ep == epochs - 1:
            hist.append((ep + 1, eval_loss(train_idx), eval_loss(test_idx) if len(test_idx) else float("nan")))
            sel = hist[-1][2] if len(test_idx) else hist[-1][1]
            if sel < best[0]:
                best = (sel, ep + 1, tr.params().cpu().numpy())
            if verbose and ((ep + 1) % (4 * check_every) == 0 or ep == epochs - 1):
                print(f"[proposal] epoch {ep + 1}: train {hist[-1][1]:.3e} test {hist[-1][2]:.3e} "
                      f"({time.perf_counter() - t0:.1f}s)", flush=True)
    params = best[2] if best[2] is not None else tr.params().cpu().numpy()
    if verbose:
        print(f"[proposal] kept the weights of epoch {best[1]} (held-out loss {best[0]:.3e})", flush=True)
    return dict(sizes=np.asarray(sizes, dtype=np.int32), params=params, out_mean=mean, out_std=std,
                n_D=np.int64(n_D), n_C=np.int64(n_C), history=np.asarray(hist, dtype=np.float64),
                n_train=np.int64(N), epochs=np.int64(epochs), seed=np.int64(seed), best_epoch=np.int64(best[1]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("pack")
    ap.add_argument("--out", required=True)
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=256)
    a = ap.parse_args()
    pack = dict(np.load(a.pack, allow_pickle=False))
    pk = train(pack, n_train=a.n_train, seed=a.seed, epochs=a.epochs, batch=a.batch)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.savez(a.out, **pk)
    print(f"[proposal] wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
