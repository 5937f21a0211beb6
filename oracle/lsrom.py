"""LS-ROM (Section 3.3) on the DD-LSPG problem with the weak FOM-port constraint, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every subdomain state is affine in its latent coordinates,
    x_i^Omega = x0_i^Omega + Phi_i^Omega xhat_i^Omega,   x_i^Gamma = x0_i^Gamma + Phi_i^Gamma xhat_i^Gamma,
(the paper's linear maps are the case x0 = 0; POD bases Phi_i = U_i(:, 1:n_i) by the energy
criterion, eq. energy_criterion).  The problem is eq. dd_lspg_NLP with an HR operator B_i
per subdomain (Section 3.1): collocation B_i = Z_i, gappy POD B_i = (Z_i Phi_i^r)^+ Z_i, or
B_i = I.  It is solved by the Lagrange-Gauss-Newton SQP method of Section 4.1 under the
same readings as rom.py (merit 0.5||F||^2 with F the KKT right-hand side, Armijo with
c1, alpha halving, relative/absolute stopping test, initial multiplier by least squares on
the first-order conditions).

This solver is deliberately written along different routes from rom.py, so that it can
check that module where the two must agree (identity activation, Section 3.3 vs 3.4):
  * the residual Jacobian with respect to the whole latent vector is formed through one
    sparse prolongation matrix per subdomain (latent vector -> global FOM state), with no
    per-block column stacking, and the sampled rows are taken by their global row ids;
  * the constraint Jacobian is the sum over subdomains of C A_i times the interface rows
    of that prolongation;
  * each SQP step is the minimiser of the QP of Lemma 2, computed by a null-space method;
    the new multiplier is the QP's multiplier, from its stationarity equations;
  * the initial multiplier solves the normal equations of the least-squares problem over
    all first-order rows with a Cholesky factorisation (the latent rows of the interior
    states do not involve lambda, so this has the same minimiser as the least-squares
    problem over the interface rows).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .burgers import BurgersFOM
from .ddmaps import DDMaps

CONVERGED, MAX_ITER, LINESEARCH_FAIL, KKT_NOT_PD, NONFINITE, STALLED = 0, 1, 2, 3, 4, 5


@dataclass
class HROperator:
    """B_i r_i = P (r[rows]) with `rows` global residual rows of subdomain i; P = None is the
    identity on those rows (collocation), a dense matrix for gappy POD."""
    rows: np.ndarray
    P: np.ndarray | None = None


def collocation_operator(grid, nodes) -> HROperator:
    """Z_i for sampled grid nodes: the r_u and r_v rows of each node (global row ids)."""
    nodes = np.asarray(nodes, dtype=np.int64)
    return HROperator(np.concatenate([nodes, nodes + grid.n_nodes]))


def gappy_pod_operator(grid, nodes, res_rows, Phi_r) -> HROperator:
    """(Z_i Phi_i^r)^+ Z_i (Section 3.1): Phi_r is the residual POD basis over the
    subdomain's residual rows `res_rows` (global ids, in that order)."""
    op = collocation_operator(grid, nodes)
    pos = {int(r): k for k, r in enumerate(res_rows)}
    ZPhi = Phi_r[[pos[int(r)] for r in op.rows]]
    return HROperator(op.rows, np.linalg.pinv(ZPhi))


@dataclass
class LSROM:
    fom: BurgersFOM
    dd: DDMaps
    C: np.ndarray                 # n_C x N_A
    x0_om: list                   # per subdomain, length N_i^Omega
    Phi_om: list                  # per subdomain, N_i^Omega x n_i^Omega
    x0_ga: list
    Phi_ga: list
    hr: list | None = None        # HROperator per subdomain; None: B_i = I

    def __post_init__(self):
        n_dof = self.dd.grid.n_dof
        self.sizes = [(P.shape[1], Q.shape[1]) for P, Q in zip(self.Phi_om, self.Phi_ga)]
        self.n_D = sum(a + b for a, b in self.sizes)
        self.n_C = self.C.shape[0]
        # Prolongation M_i: latent vector (all subdomains) -> global FOM state as seen by
        # subdomain i, x = xbase_i + M_i xhat, and the interface-row block used by the
        # constraint.  Latent layout [xhat_1^Omega; xhat_1^Gamma; xhat_2^Omega; ...].
        self.M, self.xbase, self.Mga, self.rows = [], [], [], []
        col = 0
        for i, sd in enumerate(self.dd.subdomains):
            a, b = self.sizes[i]
            xb = np.zeros(n_dof)
            xb[sd.omega] = self.x0_om[i]
            xb[sd.gamma] = self.x0_ga[i]
            r_o, c_o = np.meshgrid(sd.omega, np.arange(col, col + a), indexing="ij")
            r_g, c_g = np.meshgrid(sd.gamma, np.arange(col + a, col + a + b), indexing="ij")
            M = sp.csr_matrix((np.concatenate([self.Phi_om[i].ravel(), self.Phi_ga[i].ravel()]),
                               (np.concatenate([r_o.ravel(), r_g.ravel()]),
                                np.concatenate([c_o.ravel(), c_g.ravel()]))), shape=(n_dof, self.n_D))
            self.M.append(M)
            self.xbase.append(xb)
            self.Mga.append(M[sd.gamma])
            self.rows.append(sd.res_rows if self.hr is None else self.hr[i].rows)
            col += a + b
        self.CA = [sp.csr_matrix(self.C) @ A for A in self.dd.A]
        self.E = np.asarray(sum((CA @ Mg).toarray() for CA, Mg in zip(self.CA, self.Mga)))
        self.c0 = sum(CA @ xb[sd.gamma] for CA, xb, sd in zip(self.CA, self.xbase, self.dd.subdomains))
        self.ga_cols = np.concatenate([np.arange(o + a, o + a + b) for o, (a, b) in
                                       zip(np.cumsum([0] + [a + b for a, b in self.sizes])[:-1], self.sizes)])

    def residual(self, mu, xhat):
        """Stacked B_i r_i and its Jacobian with respect to the whole latent vector."""
        vals, jacs = [], []
        for i in range(len(self.M)):
            x = self.xbase[i] + self.M[i] @ xhat
            r = self.fom.residual(x, mu)[self.rows[i]]
            J = (self.fom.jacobian(x, mu)[self.rows[i]] @ self.M[i]).toarray()
            P = None if self.hr is None else self.hr[i].P
            if P is not None:
                r, J = P @ r, P @ J
            vals.append(r)
            jacs.append(J)
        return np.concatenate(vals), np.vstack(jacs)

    def constraint(self, xhat):
        return self.c0 + self.E @ xhat


def _kkt_residual(rom: LSROM, r, J, c, lam):
    return -np.concatenate([J.T @ r + rom.E.T @ lam, c])


def _qp_step(rom: LSROM, r, J, c):
    """Minimiser of 0.5 ||r + J s||^2 subject to c + E s = 0 (Lemma 2) and its multiplier."""
    E = rom.E
    s_p = np.linalg.lstsq(E, -c, rcond=None)[0]
    U, sv, Vt = np.linalg.svd(E)
    rank = int(np.sum(sv > sv[0] * 1e-13)) if sv.size else 0
    N = Vt[rank:].T
    y = np.linalg.lstsq(J @ N, -(r + J @ s_p), rcond=None)[0]
    s = s_p + N @ y
    lam = np.linalg.lstsq(E.T, -(J.T @ (r + J @ s)), rcond=None)[0]
    return s, lam


def _initial_multiplier(rom: LSROM, r, J):
    g = J.T @ r
    G = rom.E @ rom.E.T
    return sla.cho_solve(sla.cho_factor(G), -(rom.E @ g))


@dataclass
class LSResult:
    xhat: np.ndarray
    lam: np.ndarray
    status: int
    iters: int
    fnorm: float
    fnorm0: float


def solve(rom: LSROM, mu, xhat0=None, lam0=None, max_iter=50, tol_abs=1e-8, tol_rel=0.0, c1=1e-4,
          max_backtracks=20) -> LSResult:
    x = np.zeros(rom.n_D) if xhat0 is None else np.array(xhat0, dtype=np.float64)
    r, J = rom.residual(mu, x)
    c = rom.constraint(x)
    lam = _initial_multiplier(rom, r, J) if lam0 is None else np.array(lam0, dtype=np.float64)
    F = _kkt_residual(rom, r, J, c, lam)
    fn = float(np.linalg.norm(F))
    f0 = fn
    if not np.isfinite(fn):
        return LSResult(x, lam, NONFINITE, 0, fn, f0)
    tol = max(tol_abs, tol_rel * f0)
    for k in range(max_iter):
        if fn <= tol:
            return LSResult(x, lam, CONVERGED, k, fn, f0)
        s, lam_qp = _qp_step(rom, r, J, c)
        s_lam = lam_qp - lam
        merit0 = 0.5 * fn * fn
        alpha = 1.0
        for _ in range(max_backtracks + 1):
            xt, lt = x + alpha * s, lam + alpha * s_lam
            rt, Jt = rom.residual(mu, xt)
            ct = rom.constraint(xt)
            Ft = _kkt_residual(rom, rt, Jt, ct, lt)
            merit = 0.5 * float(Ft @ Ft)
            if np.isfinite(merit) and merit <= (1.0 - 2.0 * c1 * alpha) * merit0:
                break
            alpha *= 0.5
        else:
            return LSResult(x, lam, LINESEARCH_FAIL, k, fn, f0)
        x, lam, r, J, c, fn = xt, lt, rt, Jt, ct, float(np.sqrt(2.0 * merit))
    return LSResult(x, lam, CONVERGED if fn <= tol else MAX_ITER, max_iter, fn, f0)


def pod_maps(X_sub: np.ndarray, nu: float | None = None, n: int | None = None):
    """POD basis of a subdomain snapshot matrix (columns = snapshots): Phi = U(:, 1:n) with n
    from eq. energy_criterion (or given).  Returns (x0 = 0, Phi)."""
    U, s, _ = np.linalg.svd(X_sub, full_matrices=False)
    if n is None:
        e = np.cumsum(s ** 2)
        n = int(np.searchsorted(e, (1.0 - nu) * e[-1]) + 1)
    return np.zeros(X_sub.shape[0]), U[:, :n]
