"""Oracle: learned initial iterate for the online SQP (test infrastructure only).

The paper starts its online solves from an interpolation of training solutions over the
parameter box (Section 7.2, radial-basis interpolation of snapshot latents).  Here that role is played by a small dense
network mapping the Burgers parameters (a, lambda) to every subdomain's latents and the
multipliers, trained on converged solves of the method itself.  This module is the plain
FP64 statement of that network, its gradient and its optimiser, plus the rule that keeps
the method's own zero start whenever the proposal is worse.  Only the tests, the smoke
check and the CPU baseline of the benchmark import it.

Definitions (readings of what the paper leaves open):
  * inputs  (log10 a, lambda), each mapped affinely onto [-1, 1] over the parameter box
    a in [1, 1e4], lambda in [5, 20];
  * layers  2 -> 256 -> 256 -> n_D + n_C, SiLU on the hidden layers, linear output;
  * targets the converged [xhat; lambda] of each training solve, standardised per
    component with the training-set mean and standard deviation (a deviation below
    1e-12 is replaced by 1);
  * loss    mean squared error over the minibatch and all components;
  * Adam    (0.9, 0.999, 1e-8), learning rate 1e-3, Glorot-uniform weights, zero biases;
  * fallback  the first KKT residual norm ||F(proposal)|| is compared with the zero-start
    norm ||F(0, lambda_LS)||; the solve starts from the zero start when the proposal's is
    larger, so the start it uses never has a larger first residual than the zero start.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LOG_A_RANGE = (0.0, 4.0)
LAM_RANGE = (5.0, 20.0)


def encode_inputs(mu: np.ndarray) -> np.ndarray:
    """(a, lambda) [B][2] -> network inputs [B][2] in [-1, 1]."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    la = np.log10(mu[:, 0])
    u0 = 2.0 * (la - LOG_A_RANGE[0]) / (LOG_A_RANGE[1] - LOG_A_RANGE[0]) - 1.0
    u1 = 2.0 * (mu[:, 1] - LAM_RANGE[0]) / (LAM_RANGE[1] - LAM_RANGE[0]) - 1.0
    return np.stack([u0, u1], axis=1)


def silu(z: np.ndarray) -> np.ndarray:
    return z / (1.0 + np.exp(-z))


def silu_prime(z: np.ndarray) -> np.ndarray:
    s = 1.0 / (1.0 + np.exp(-z))
    return s + z * s * (1.0 - s)


@dataclass
class Standardiser:
    mean: np.ndarray
    std: np.ndarray

    def forward(self, Y: np.ndarray) -> np.ndarray:
        return (Y - self.mean) / self.std

    def inverse(self, Yn: np.ndarray) -> np.ndarray:
        return Yn * self.std + self.mean


def standardiser(Y: np.ndarray) -> Standardiser:
    m = Y.mean(axis=0)
    s = Y.std(axis=0)
    s = np.where(s < 1e-12, 1.0, s)
    return Standardiser(m, s)


@dataclass
class MLP:
    """Dense network; layers[k] = (W [out][in], b [out]).  SiLU after every layer but the last."""
    layers: list

    @property
    def sizes(self):
        return [self.layers[0][0].shape[1]] + [W.shape[0] for W, _ in self.layers]

    def params(self) -> list:
        out = []
        for W, b in self.layers:
            out += [W, b]
        return out

    def forward(self, X: np.ndarray, keep: bool = False):
        """Network output for inputs X [B][in]; with keep=True also the layer inputs and
        pre-activations needed by the gradient."""
        A = np.asarray(X, dtype=np.float64)
        cache = []
        L = len(self.layers)
        for k, (W, b) in enumerate(self.layers):
            Z = A @ W.T + b
            cache.append((A, Z))
            A = silu(Z) if k < L - 1 else Z
        return (A, cache) if keep else A

    def loss_and_grad(self, X: np.ndarray, T: np.ndarray):
        """Mean squared error against targets T and its gradient, by the chain rule layer
        by layer (backward through the linear maps and the SiLU)."""
        Y, cache = self.forward(X, keep=True)
        R = Y - T
        loss = float(np.mean(R * R))
        dA = 2.0 * R / R.size
        grads = [None] * (2 * len(self.layers))
        for k in range(len(self.layers) - 1, -1, -1):
            A_in, Z = cache[k]
            W, _ = self.layers[k]
            dZ = dA if k == len(self.layers) - 1 else dA * silu_prime(Z)
            grads[2 * k] = dZ.T @ A_in
            grads[2 * k + 1] = dZ.sum(axis=0)
            dA = dZ @ W
        return loss, grads


def mlp_from_init(init: list) -> MLP:
    return MLP([(np.array(W, dtype=np.float64), np.array(b, dtype=np.float64)) for W, b in init])


@dataclass
class ProposalReport:
    epochs: int
    train_loss: float
    test_loss: float
    history: list = field(default_factory=list)


def train_proposal(net: MLP, Xin: np.ndarray, Tn: np.ndarray, train_idx: np.ndarray, test_idx: np.ndarray,
                   epochs: int, batch: int, seed: int, lr: float = 1e-3, order_fn=None) -> ProposalReport:
    """Adam on minibatches of the training rows; order_fn(n, seed, epoch) gives each epoch's
    visiting order of the training rows."""
    from .autoencoder import Adam
    opt = Adam(net.params(), lr=lr)
    hist = []
    for ep in range(epochs):
        order = train_idx[order_fn(len(train_idx), seed, ep)]
        for s0 in range(0, len(order), batch):
            rows = order[s0:s0 + batch]
            _, g = net.loss_and_grad(Xin[rows], Tn[rows])
            opt.step(net.params(), g)
        hist.append(float(np.mean((net.forward(Xin[train_idx]) - Tn[train_idx]) ** 2)))
    te = float(np.mean((net.forward(Xin[test_idx]) - Tn[test_idx]) ** 2)) if len(test_idx) else float("nan")
    return ProposalReport(epochs, hist[-1] if hist else float("nan"), te, hist)


def propose(net: MLP, st: Standardiser, mu: np.ndarray, n_D: int):
    """Proposed (xhat0 [B][n_D], lambda0 [B][n_C]) for parameters mu [B][2]."""
    Y = st.inverse(net.forward(encode_inputs(mu)))
    return Y[:, :n_D], Y[:, n_D:]


def use_zero_start(f_proposal: float, f_zero: float) -> bool:
    """The fallback rule: keep the zero start when the proposal's first residual is larger
    (a non-finite proposal residual also falls back)."""
    return not (np.isfinite(f_proposal) and f_proposal <= f_zero)
