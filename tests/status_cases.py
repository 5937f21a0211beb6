"""Model packs whose SQP must stop on a failure status (shared by the oracle pins and the
GPU status tests).  Each construction makes a hypothesis of Lemma 1 fail exactly, so that
the failure does not depend on rounding:
  * a zero row of C: the constraint Jacobian has an exactly zero row (no full row rank);
  * a zero column of an interior decoder's W1: that latent has no effect, so Z R_i has an
    exactly zero column and H_i an exactly zero row and column (not positive definite)."""
import numpy as np


def rank_deficient_constraint(pack: dict, row: int = 0) -> dict:
    p = dict(pack)
    C = np.array(p["C"], dtype=np.float64)
    C[row] = 0.0
    p["C"] = C
    return p


def singular_block(pack: dict, sd: int = 0, col: int = 1) -> dict:
    p = dict(pack)
    W1 = np.array(p[f"om{sd}_W1"], dtype=np.float64)
    W1[:, col] = 0.0
    p[f"om{sd}_W1"] = W1
    return p
