"""Shallow, wide, band-masked autoencoders (Sections 3.4, 5.1 and 7.3), FP64.

Architecture (eq. autoencoder_architecture):
    encoder h(x)    = W2^h sigma(W1^h x~ + b1^h)          (no output bias)
    decoder g(xhat) = x_ref + W2^g sigma(W1^g xhat + b1^g)
with W2^g (N x w) carrying the three-band mask and W1^h (w x N) its transpose; the
other weights are dense.  x~ = (x - m) / s is the [-1, 1] normalisation of the
snapshots; the de-normalisation layer is folded into the decoder at export
(rows of W2^g scaled by s, x_ref = m), which keeps the mask.

Three-band mask (Section 7.3): row r has b contiguous nonzeros in each of three bands;
the bands shift right by s columns per row and are b*s columns apart.  Reading: band
k in {-1, 0, 1} of row r covers columns [r s + k b s, r s + k b s + b) intersected with
[0, w), with width w = N s.  This reproduces the paper's widths and nonzero counts.

Training follows Section 7.3 and eq. autoencoder_AbsMSE_loss: MSE in the raw state
space averaged over the minibatch, Adam, reduce-on-plateau, early stopping.  Readings:
Adam betas (0.9, 0.999), eps 1e-8, plateau factor 0.1; Glorot-uniform init with
masked layers using their mean nonzeros per row/column as fan-in/fan-out.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

import seeded_inputs as si

ACT_SIGMOID, ACT_SWISH, ACT_IDENTITY = 0, 1, 2


def act(z: np.ndarray, kind: int):
    """Activation value and derivative."""
    if kind == ACT_SIGMOID:
        s = 1.0 / (1.0 + np.exp(-z))
        return s, s * (1.0 - s)
    if kind == ACT_SWISH:
        s = 1.0 / (1.0 + np.exp(-z))
        return z * s, s + z * s * (1.0 - s)
    if kind == ACT_IDENTITY:
        return z.copy(), np.ones_like(z)
    raise ValueError(kind)


def band_columns(N: int, b: int, s: int):
    """Column index of every mask slot [N, 3, b] and its validity (inside [0, w))."""
    w = N * s
    r = np.arange(N)[:, None, None]
    k = np.arange(-1, 2)[None, :, None]
    t = np.arange(b)[None, None, :]
    cols = r * s + k * b * s + t
    return cols, (cols >= 0) & (cols < w)


def band_mask(N: int, b: int, s: int) -> sp.csr_matrix:
    """0/1 pattern of the decoder output layer W2^g (N x N s)."""
    cols, valid = band_columns(N, b, s)
    rows = np.broadcast_to(np.arange(N)[:, None, None], cols.shape)
    return sp.csr_matrix((np.ones(valid.sum()), (rows[valid], cols[valid])), shape=(N, N * s))


def parameter_count(N: int, n: int, b: int, s: int) -> int:
    """Trainable parameters of one autoencoder: two masked layers, two dense layers, two
    hidden biases, no output biases."""
    nnz = int(band_mask(N, b, s).nnz)
    w = N * s
    return 2 * nnz + 2 * w + 2 * n * w


@dataclass
class Decoder:
    """Exported decoder g(xhat) = x_ref + W2 sigma(W1 xhat + b1), W2 stored as band values."""
    W1: np.ndarray        # [w, n]
    b1: np.ndarray        # [w]
    W2vals: np.ndarray    # [N, 3, b]; zero in slots outside [0, w)
    x_ref: np.ndarray     # [N]
    b: int
    s: int
    act: int

    @property
    def N(self):
        return self.x_ref.shape[0]

    @property
    def n(self):
        return self.W1.shape[1]

    @property
    def w(self):
        return self.W1.shape[0]

    def W2(self) -> sp.csr_matrix:
        cols, valid = band_columns(self.N, self.b, self.s)
        rows = np.broadcast_to(np.arange(self.N)[:, None, None], cols.shape)
        return sp.csr_matrix((self.W2vals[valid], (rows[valid], cols[valid])), shape=(self.N, self.w))


def decode(dec: Decoder, xhat: np.ndarray) -> np.ndarray:
    z = dec.W1 @ xhat + dec.b1
    a, _ = act(z, dec.act)
    return dec.x_ref + dec.W2() @ a


def decode_jacobian(dec: Decoder, xhat: np.ndarray):
    """g(xhat) and dg/dxhat = W2 diag(sigma'(z)) W1 (N x n)."""
    z = dec.W1 @ xhat + dec.b1
    a, da = act(z, dec.act)
    W2 = dec.W2()
    return dec.x_ref + W2 @ a, W2 @ (da[:, None] * dec.W1)


# ----------------------------------------------------------------------------------
# Training
# ----------------------------------------------------------------------------------

@dataclass
class AEParams:
    W1e: np.ndarray   # values of the transposed-mask encoder layer (CSR data order of maskT)
    b1e: np.ndarray   # [w]
    W2e: np.ndarray   # [n, w]
    W1d: np.ndarray   # [w, n]
    b1d: np.ndarray   # [w]
    W2d: np.ndarray   # values of the decoder mask (CSR data order of mask)

    def as_list(self):
        return [self.W1e, self.b1e, self.W2e, self.W1d, self.b1d, self.W2d]


@dataclass
class Normalisation:
    m: np.ndarray
    s: np.ndarray


def normalisation(X: np.ndarray) -> Normalisation:
    """Per-component min-max map onto [-1, 1] (Section 7.3).  X is [n_snap, N].
    Components with (numerically) no range keep scale 1."""
    mx, mn = X.max(0), X.min(0)
    m = 0.5 * (mx + mn)
    s = 0.5 * (mx - mn)
    s = np.where(s < 1e-14 * np.maximum(1.0, np.abs(m)), 1.0, s)
    return Normalisation(m, s)


class MaskedAE:
    """Autoencoder with hand-written forward/backward passes over a minibatch."""

    def __init__(self, N: int, n: int, b: int, s: int, activation: int):
        self.N, self.n, self.b, self.s, self.act = N, n, b, s, activation
        self.w = N * s
        self.mask = band_mask(N, b, s)                 # N x w (decoder output layer)
        self.maskT = self.mask.T.tocsr()               # w x N (encoder input layer)
        self.mask.sort_indices()
        self.maskT.sort_indices()
        # row/col of every stored entry, for the masked weight gradients
        self.m_rows = np.repeat(np.arange(N), np.diff(self.mask.indptr))
        self.m_cols = self.mask.indices.copy()
        self.mT_rows = np.repeat(np.arange(self.w), np.diff(self.maskT.indptr))
        self.mT_cols = self.maskT.indices.copy()

    def init_params(self, seed: int) -> AEParams:
        seeds = si.spawn_seeds(seed, 6)
        nnz = self.mask.nnz
        per_row = nnz / self.N
        per_col = nnz / self.w
        W1e = si.glorot_uniform(per_col, per_row, (nnz,), si.rng(seeds[0]))
        W2e = si.glorot_uniform(self.w, self.n, (self.n, self.w), si.rng(seeds[2]))
        W1d = si.glorot_uniform(self.n, self.w, (self.w, self.n), si.rng(seeds[3]))
        W2d = si.glorot_uniform(per_row, per_col, (nnz,), si.rng(seeds[5]))
        return AEParams(W1e, np.zeros(self.w), W2e, W1d, np.zeros(self.w), W2d)

    def _enc_mat(self, p: AEParams):
        return sp.csr_matrix((p.W1e, self.maskT.indices, self.maskT.indptr), shape=(self.w, self.N))

    def _dec_mat(self, p: AEParams):
        return sp.csr_matrix((p.W2d, self.mask.indices, self.mask.indptr), shape=(self.N, self.w))

    def encode(self, p: AEParams, Xn: np.ndarray) -> np.ndarray:
        """Latents of normalised snapshots Xn [B, N]."""
        ze = (self._enc_mat(p) @ Xn.T).T + p.b1e
        ae, _ = act(ze, self.act)
        return ae @ p.W2e.T

    def forward_backward(self, p: AEParams, Xn: np.ndarray, scale: np.ndarray):
        """Loss (1/B) sum ||scale o (Xn - Y)||^2 and its gradients (raw-space MSE)."""
        B = Xn.shape[0]
        E1 = self._enc_mat(p)
        D2 = self._dec_mat(p)
        ze = (E1 @ Xn.T).T + p.b1e                   # [B, w]
        ae, dae = act(ze, self.act)
        xh = ae @ p.W2e.T                            # [B, n]
        zd = xh @ p.W1d.T + p.b1d                    # [B, w]
        ad, dad = act(zd, self.act)
        Y = (D2 @ ad.T).T                            # [B, N]
        diff = (Y - Xn) * scale
        loss = float((diff * diff).sum() / B)
        dY = (2.0 / B) * diff * scale                # dL/dY
        gW2d = np.einsum("bk,bk->k", dY[:, self.m_rows], ad[:, self.m_cols])
        dzd = (D2.T @ dY.T).T * dad
        gW1d = dzd.T @ xh
        gb1d = dzd.sum(0)
        dxh = dzd @ p.W1d
        gW2e = dxh.T @ ae
        dze = (dxh @ p.W2e) * dae
        gW1e = np.einsum("bk,bk->k", dze[:, self.mT_rows], Xn[:, self.mT_cols])
        gb1e = dze.sum(0)
        return loss, AEParams(gW1e, gb1e, gW2e, gW1d, gb1d, gW2d)

    def loss(self, p: AEParams, Xn: np.ndarray, scale: np.ndarray) -> float:
        xh = self.encode(p, Xn)
        zd = xh @ p.W1d.T + p.b1d
        ad, _ = act(zd, self.act)
        Y = (self._dec_mat(p) @ ad.T).T
        diff = (Y - Xn) * scale
        return float((diff * diff).sum() / Xn.shape[0])


class Adam:
    def __init__(self, params: list, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(x) for x in params]
        self.v = [np.zeros_like(x) for x in params]
        self.t = 0

    def step(self, params: list, grads: list):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for x, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            x -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


@dataclass
class TrainReport:
    epochs: int
    train_loss: float
    test_loss: float
    history: list = field(default_factory=list)


def train(ae: MaskedAE, X: np.ndarray, seed: int, epochs: int, batch: int = 32, lr: float = 1e-3,
          test_frac: float = 0.1, plateau_patience: int = 50, stop_patience: int = 300,
          verbose: bool = False):
    """Train on raw snapshots X [n_snap, N]; returns (params, normalisation, report)."""
    g = si.rng(seed)
    n_snap = X.shape[0]
    perm = g.permutation(n_snap)
    n_test = max(1, int(round(test_frac * n_snap))) if n_snap > 1 else 0
    test_idx, train_idx = perm[:n_test], perm[n_test:]
    nm = normalisation(X[train_idx])
    Xn = (X - nm.m) / nm.s
    p = ae.init_params(int(g.integers(0, 2 ** 62)))
    opt = Adam(p.as_list(), lr=lr)
    best, best_p, since_best, since_plateau, plateau_best = np.inf, None, 0, 0, np.inf
    hist = []
    tr_loss = te_loss = np.nan
    ep = 0
    for ep in range(1, epochs + 1):
        order = g.permutation(train_idx)
        tot = 0.0
        for k in range(0, len(order), batch):
            idx = order[k:k + batch]
            loss, grads = ae.forward_backward(p, Xn[idx], nm.s)
            opt.step(p.as_list(), grads.as_list())
            tot += loss * len(idx)
        tr_loss = tot / len(order)
        te_loss = ae.loss(p, Xn[test_idx], nm.s) if n_test else tr_loss
        hist.append((tr_loss, te_loss))
        if te_loss < plateau_best:
            plateau_best, since_plateau = te_loss, 0
        else:
            since_plateau += 1
            if since_plateau > plateau_patience:
                opt.lr *= 0.1
                since_plateau = 0
                plateau_best = te_loss
        if te_loss < best:
            best, since_best = te_loss, 0
            best_p = AEParams(*[x.copy() for x in p.as_list()])
        else:
            since_best += 1
            if since_best > stop_patience:
                break
        if verbose and ep % 50 == 0:
            print(f"  epoch {ep}: train {tr_loss:.3e} test {te_loss:.3e} lr {opt.lr:.1e}", flush=True)
    return best_p, nm, TrainReport(ep, tr_loss, best, hist)


def export_decoder(ae: MaskedAE, p: AEParams, nm: Normalisation, center: np.ndarray | None = None) -> Decoder:
    """Fold the de-normalisation into the decoder.  If `center` (a latent vector) is
    given, the latent coordinate is shifted so that xhat = 0 decodes what `center` did
    (b1 <- b1 + W1 center); the trial manifold is unchanged."""
    cols, valid = band_columns(ae.N, ae.b, ae.s)
    vals = np.zeros(cols.shape)
    # CSR data of the mask is ordered by (row, col) ascending, which is also the order of
    # the valid slots of band_columns (bands ascending, columns ascending inside a band).
    vals[valid] = p.W2d
    vals *= nm.s[:, None, None]
    b1 = p.b1d.copy()
    if center is not None:
        b1 = b1 + p.W1d @ center
    return Decoder(p.W1d.copy(), b1, vals, nm.m.copy(), ae.b, ae.s, ae.act)
