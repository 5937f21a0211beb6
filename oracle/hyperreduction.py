"""Collocation hyper-reduction and decoder subnets (Sections 3.3, 5.3, 5.4).

* pod_basis: thin SVD with the energy criterion (eq. energy_criterion).
* greedy_sample: row-sampling Z_i for collocation HR.  The paper cites the greedy
  procedure of Carlberg et al. (2013, Alg. 3) without printing it.  Reading used here
  (parity unpinned; pinned only by invariants): the sampling unit is a grid node (its
  r_u and r_v rows).  Basis vectors of the residual POD basis are visited in order,
  cycling, until the requested number of nodes is chosen.  For vector k the
  gappy-POD least-squares fit of phi_k on the rows chosen so far, using the vectors
  visited before it in the current cycle, is formed; the unchosen node whose two rows
  carry the largest squared fit error is added (ties: lowest node id).
* subnet: index sets I_o, I_h and the sliced weights of eq. subnet.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .autoencoder import Decoder, act, band_columns


def pod_basis(X: np.ndarray, tol: float) -> np.ndarray:
    """Columns of U from the thin SVD of X [N, n_snap]: the smallest n with
    sum_{j<=n} sigma_j^2 >= (1 - tol) sum_j sigma_j^2."""
    U, S, _ = np.linalg.svd(X, full_matrices=False)
    e = S ** 2
    tot = e.sum()
    if tot == 0.0:
        return U[:, :1]
    cum = np.cumsum(e)
    n = int(np.searchsorted(cum, (1.0 - tol) * tot) + 1)
    return U[:, :min(n, U.shape[1])]


def greedy_sample(Phi: np.ndarray, n_own: int, n_nodes: int) -> np.ndarray:
    """Choose n_nodes of the n_own local nodes.  Phi has 2*n_own rows: rows [0, n_own)
    are the r_u rows and rows [n_own, 2 n_own) the r_v rows of the same nodes.
    Returns local node positions, ascending."""
    n_nodes = min(n_nodes, n_own)
    nr = Phi.shape[1]
    chosen: list[int] = []
    taken = np.zeros(n_own, dtype=bool)
    step = 0
    while len(chosen) < n_nodes:
        k = step % nr
        phi = Phi[:, k]
        if k == 0 or not chosen:
            err = phi
        else:
            rows = np.concatenate([np.array(chosen), np.array(chosen) + n_own])
            basis = Phi[:, :k]
            c, *_ = np.linalg.lstsq(basis[rows], phi[rows], rcond=None)
            err = phi - basis @ c
        score = err[:n_own] ** 2 + err[n_own:] ** 2
        score[taken] = -1.0
        j = int(np.argmax(score))          # argmax returns the lowest index on ties
        chosen.append(j)
        taken[j] = True
        step += 1
    return np.array(sorted(chosen), dtype=np.int64)


@dataclass
class Subnet:
    I_o: np.ndarray      # output rows kept (ascending)
    I_h: np.ndarray      # hidden units kept (ascending)
    W1: np.ndarray       # [|I_h|, n]   rows of W1
    b1: np.ndarray       # [|I_h|]
    W2: np.ndarray       # [|I_o|, |I_h|] dense slice of W2 (mostly zero)
    x_ref: np.ndarray    # [|I_o|]
    act: int


def subnet(dec: Decoder, I_o: np.ndarray) -> Subnet:
    """eq. subnet: I_h = {j : exists i in I_o with (W2)_ij in the mask};
    W2~ = W2[I_o, I_h], W1~ = W1[I_h, :], b1~ = b1[I_h].  The de-normalisation offset
    x_ref[I_o] is carried along."""
    cols, valid = band_columns(dec.N, dec.b, dec.s)
    I_o = np.asarray(sorted(set(int(i) for i in I_o)), dtype=np.int64)
    I_h = np.unique(cols[I_o][valid[I_o]])
    W2 = dec.W2().tocsr()[I_o][:, I_h].toarray()
    return Subnet(I_o, I_h, dec.W1[I_h].copy(), dec.b1[I_h].copy(), W2, dec.x_ref[I_o].copy(), dec.act)


def subnet_decode(sn: Subnet, xhat: np.ndarray):
    z = sn.W1 @ xhat + sn.b1
    a, da = act(z, sn.act)
    return sn.x_ref + sn.W2 @ a, sn.W2 @ (da[:, None] * sn.W1)
