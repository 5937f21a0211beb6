"""DD-LSPG ROM with weak FOM-port constraints and collocation HR, solved by the
Lagrange-Gauss-Newton SQP method (Sections 3.1, 4.1; eqs. dd_lspg_NLP,
dd_lspg_NLP_general, optimality_residuals, sqp_system, gauss_newton_hessian,
sqp_update), FP64.

Everything here is the plain definition:
  * the decoders are evaluated in full and the subdomain residual r_i is evaluated on
    the whole grid through eq. subdomain_residual_def, then the collocation operator
    B_i = Z_i keeps the rows of the sampled nodes;
  * R_i = [dr_i/dx^Omega dg^Omega/dxhat^Omega, dr_i/dx^Gamma dg^Gamma/dxhat^Gamma];
  * H_i = (Z R_i)^T (Z R_i), rho_i = (Z R_i)^T Z r_i + E_i^T lambda,
    E_i = [0, C A_i dg^Gamma/dxhat^Gamma], constraint sum_i C A_i g_i^Gamma;
  * the KKT matrix of eq. sqp_system is assembled densely and solved with LAPACK
    (numpy.linalg.solve); no Schur complement, no blocking.

Readings (the paper leaves these open): the line search merit is
phi(alpha) = 0.5 ||F(xhat + alpha s, lambda + alpha s_lambda)||^2 with F the KKT
right-hand side; a step is accepted when phi(alpha) <= (1 - 2 c1 alpha) phi(0),
c1 = 1e-4, alpha halving, at most `max_backtracks` halvings; otherwise the solve stops
with status LINESEARCH_FAIL at the last accepted point.  The solve stops when
||F||_2 <= max(tol_abs, tol_rel ||F_0||_2) or after max_iter steps.  The initial
multiplier is the least-squares solution of the interface rows of the first-order
conditions (eq. optimality_residuals b) at the initial latents.  A step is taken only
where Lemma 1's hypotheses hold (every H_i positive definite, the constraint Jacobian of
full row rank); otherwise the solve stops with KKT_NOT_PD.  Where the constraint Jacobian
at the start lacks full row rank the least-squares multiplier is not unique: the solve
stops at once with KKT_NOT_PD and lambda = 0.  A start whose KKT residual is not finite
stops with NONFINITE.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .autoencoder import Decoder, decode_jacobian, decode
from .burgers import BurgersFOM, Grid
from .ddmaps import DDMaps, build_dd, subdomain_residual_jac

CONVERGED, MAX_ITER, LINESEARCH_FAIL, KKT_NOT_PD, NONFINITE, STALLED = 0, 1, 2, 3, 4, 5


@dataclass
class ROMModel:
    grid: Grid
    nsx: int
    nsy: int
    dec_om: list            # Decoder per subdomain (interior)
    dec_ga: list            # Decoder per subdomain (interface)
    hr_nodes: list | None   # sampled global node ids per subdomain (None: B_i = I)
    C: np.ndarray           # n_C x N_A (weak FOM-port constraint); unused when A_hat is given
    dd: DDMaps = None
    fom: BurgersFOM = None
    CA: list = None
    A_hat: list | None = None   # strong ROM-port constraint: sum_i A_hat[i] xhat_i^Gamma = 0

    def __post_init__(self):
        if self.dd is None:
            self.dd = build_dd(self.grid, self.nsx, self.nsy)
        if self.fom is None:
            self.fom = BurgersFOM(self.grid)
        self.CA = None if self.A_hat is not None else [self.C @ A.toarray() for A in self.dd.A]
        self._zrows = []
        for i, sd in enumerate(self.dd.subdomains):
            n_own = len(sd.own_nodes)
            if self.hr_nodes is None:
                self._zrows.append(np.arange(2 * n_own))
            else:
                loc = np.searchsorted(sd.own_nodes, np.asarray(self.hr_nodes[i]))
                if not np.array_equal(sd.own_nodes[loc], np.asarray(self.hr_nodes[i])):
                    raise ValueError("HR nodes must be owned by their subdomain")
                self._zrows.append(np.concatenate([loc, loc + n_own]))

    @property
    def n_sub(self):
        return len(self.dec_om)

    @property
    def n_C(self):
        return self.A_hat[0].shape[0] if self.A_hat is not None else self.C.shape[0]

    def sizes(self):
        return [(d.n, e.n) for d, e in zip(self.dec_om, self.dec_ga)]

    @property
    def n_D(self):
        return sum(a + b for a, b in self.sizes())

    def offsets(self):
        off, o = [], 0
        for a, b in self.sizes():
            off.append(o)
            o += a + b
        return off

    def split(self, xhat):
        """xhat = [xhat_1^Omega; xhat_1^Gamma; ...] (eq. sqp_notation) -> per-subdomain pairs."""
        out = []
        for o, (a, b) in zip(self.offsets(), self.sizes()):
            out.append((xhat[o:o + a], xhat[o + a:o + a + b]))
        return out


@dataclass
class Evaluation:
    H: list          # H_i  (n_i x n_i)
    g: list          # (Z R_i)^T Z r_i  (n_i)
    EG: list         # C A_i dg^Gamma/dxhat^Gamma  (n_C x n_i^Gamma)
    c: np.ndarray    # sum_i C A_i g_i^Gamma
    Zr: list
    ZR: list


def _decode_jac(dec, x):
    """Value and Jacobian of a decoder: a banded one (autoencoder.Decoder) or an interface
    decoder assembled from port decoders (srpc.PortInterfaceDecoder)."""
    return dec.decode_jacobian(x) if hasattr(dec, "decode_jacobian") else decode_jacobian(dec, x)


def _decode(dec, x):
    return dec.decode(x) if hasattr(dec, "decode") else decode(dec, x)


def evaluate(model: ROMModel, mu, xhat: np.ndarray) -> Evaluation:
    """Per-subdomain SQP quantities at xhat (no multiplier terms).  Weak FOM-port constraint:
    c = sum_i C A_i g_i^Gamma, E_i^Gamma = C A_i dg_i^Gamma/dxhat; strong ROM-port constraint:
    c = sum_i Ahat_i xhat_i^Gamma, E_i^Gamma = Ahat_i."""
    H, g, EG, Zr_l, ZR_l = [], [], [], [], []
    c = np.zeros(model.n_C)
    for i, (xo, xg) in enumerate(model.split(xhat)):
        go, Jo = _decode_jac(model.dec_om[i], xo)
        gg, Jg = _decode_jac(model.dec_ga[i], xg)
        r, dro, drg = subdomain_residual_jac(model.fom, model.dd, i, go, gg, mu)
        z = model._zrows[i]
        Zr = r[z]
        ZR = np.hstack([dro[z] @ Jo, drg[z] @ Jg])
        H.append(ZR.T @ ZR)
        g.append(ZR.T @ Zr)
        if model.A_hat is not None:
            EG.append(model.A_hat[i].copy())
            c += model.A_hat[i] @ xg
        else:
            EG.append(model.CA[i] @ Jg)
            c += model.CA[i] @ gg
        Zr_l.append(Zr)
        ZR_l.append(ZR)
    return Evaluation(H, g, EG, c, Zr_l, ZR_l)


def kkt_rhs(model: ROMModel, ev: Evaluation, lam: np.ndarray) -> np.ndarray:
    """F(xhat, lambda) = -[rho_1; ...; rho_n; sum_i Atilde_i]."""
    parts = []
    for i, (a, b) in enumerate(model.sizes()):
        rho = ev.g[i].copy()
        rho[a:] += ev.EG[i].T @ lam
        parts.append(rho)
    parts.append(ev.c)
    return -np.concatenate(parts)


def kkt_matrix(model: ROMModel, ev: Evaluation) -> np.ndarray:
    nD, nC = model.n_D, model.n_C
    K = np.zeros((nD + nC, nD + nC))
    for i, (o, (a, b)) in enumerate(zip(model.offsets(), model.sizes())):
        K[o:o + a + b, o:o + a + b] = ev.H[i]
        K[nD:, o + a:o + a + b] = ev.EG[i]
        K[o + a:o + a + b, nD:] = ev.EG[i].T
    return K


def kkt_step(model: ROMModel, ev: Evaluation, lam: np.ndarray):
    """Solve eq. sqp_system; returns (s_x, s_lambda)."""
    sol = np.linalg.solve(kkt_matrix(model, ev), kkt_rhs(model, ev, lam))
    return sol[:model.n_D], sol[model.n_D:]


def initial_multiplier(model: ROMModel, ev: Evaluation) -> np.ndarray:
    """argmin_lambda || [ g_i^Gamma + (E_i^Gamma)^T lambda ]_i ||_2."""
    rows, rhs = [], []
    for i, (a, b) in enumerate(model.sizes()):
        rows.append(ev.EG[i].T)
        rhs.append(-ev.g[i][a:])
    lam, *_ = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)
    return lam


def blocks_positive_definite(ev: Evaluation) -> bool:
    """First hypothesis of Lemma 1: every H_i is positive definite (LAPACK Cholesky succeeds)."""
    try:
        for Hi in ev.H:
            np.linalg.cholesky(Hi)
        return True
    except np.linalg.LinAlgError:
        return False


def constraint_full_row_rank(model: ROMModel, ev: Evaluation) -> bool:
    """Second hypothesis of Lemma 1: the constraint Jacobian [E_1, ..., E_n] (only interface
    columns are nonzero) has full row rank n_C; numerical rank by SVD with numpy's default
    threshold."""
    if model.n_C == 0:
        return True
    return int(np.linalg.matrix_rank(np.hstack(ev.EG))) == model.n_C


def start_multiplier(model: ROMModel, ev: Evaluation):
    """The initial multiplier and whether it is defined: the least-squares multiplier when the
    constraint Jacobian has full row rank; otherwise the least-squares problem has no unique
    solution (and Lemma 1 fails), lambda = 0 is returned with False."""
    if not constraint_full_row_rank(model, ev):
        return np.zeros(model.n_C), False
    return initial_multiplier(model, ev), True


@dataclass
class SQPOptions:
    max_iter: int = 50
    tol_abs: float = 1e-8
    tol_rel: float = 0.0
    c1: float = 1e-4
    max_backtracks: int = 20
    stall_tol: float = 0.0    # > 0: an Armijo failure with ||F|| <= stall_tol ||F_0|| stops with STALLED
    stall_ratio: float = 0.0  # > 0 (with stall_tol): an accepted step ending above the tolerance at
    #                           ||F|| <= stall_tol ||F_0|| with ||F_new|| > stall_ratio ||F_old|| stops with STALLED


@dataclass
class SQPResult:
    xhat: np.ndarray
    lam: np.ndarray
    status: int
    iters: int
    fnorm: float
    fnorm0: float
    evaluations: int
    history: list = field(default_factory=list)


def sqp_step(model: ROMModel, mu, xhat, lam, opts: SQPOptions, ev: Evaluation | None = None, f0: float = np.inf):
    """One Lagrange-Gauss-Newton SQP iteration from (xhat, lambda): KKT step, then
    Armijo backtracking.  Returns (xhat+, lambda+, ev+, ||F+||, status, n_evals, alpha);
    status is -1 for an accepted step."""
    if ev is None:
        ev = evaluate(model, mu, xhat)
    if not (blocks_positive_definite(ev) and constraint_full_row_rank(model, ev)):
        return xhat, lam, ev, np.linalg.norm(kkt_rhs(model, ev, lam)), KKT_NOT_PD, 0, 0.0
    F = kkt_rhs(model, ev, lam)
    phi0 = 0.5 * float(F @ F)
    sx, sl = kkt_step(model, ev, lam)
    alpha = 1.0
    for nb in range(opts.max_backtracks + 1):
        xt, lt = xhat + alpha * sx, lam + alpha * sl
        evt = evaluate(model, mu, xt)
        Ft = kkt_rhs(model, evt, lt)
        phi = 0.5 * float(Ft @ Ft)
        if not np.isfinite(phi):
            pass
        elif phi <= (1.0 - 2.0 * opts.c1 * alpha) * phi0:
            return xt, lt, evt, np.sqrt(2.0 * phi), -1, nb + 1, alpha
        if np.sqrt(2.0 * phi0) <= opts.stall_tol * f0:
            return xhat, lam, ev, np.sqrt(2.0 * phi0), STALLED, nb + 1, 0.0
        alpha *= 0.5
    return xhat, lam, ev, np.sqrt(2.0 * phi0), LINESEARCH_FAIL, opts.max_backtracks + 1, 0.0


def sqp_solve(model: ROMModel, mu, xhat0: np.ndarray | None = None, lam0: np.ndarray | None = None,
              opts: SQPOptions = SQPOptions(), f_ref: float | None = None) -> SQPResult:
    """SQP from (xhat0, lam0) (zero latents and the least-squares multiplier by default).
    The relative tolerance and the stagnation test are taken relative to f_ref, by default
    the first KKT residual norm of this start."""
    x = np.zeros(model.n_D) if xhat0 is None else np.array(xhat0, dtype=np.float64)
    ev = evaluate(model, mu, x)
    lam_ok = True
    if lam0 is None:
        lam, lam_ok = start_multiplier(model, ev)
    else:
        lam = np.array(lam0, dtype=np.float64)
    F = kkt_rhs(model, ev, lam)
    fn = float(np.linalg.norm(F))
    f0 = fn if f_ref is None else float(f_ref)
    n_eval = 1
    hist = [fn]
    if not np.isfinite(fn):
        return SQPResult(x, lam, NONFINITE, 0, fn, f0, n_eval, hist)
    if not lam_ok:
        return SQPResult(x, lam, KKT_NOT_PD, 0, fn, f0, n_eval, hist)
    tol = max(opts.tol_abs, opts.tol_rel * f0)
    for k in range(opts.max_iter):
        if fn <= tol:
            return SQPResult(x, lam, CONVERGED, k, fn, f0, n_eval, hist)
        fn_old = fn
        x, lam, ev, fn, st, ne, _ = sqp_step(model, mu, x, lam, opts, ev, f0)
        n_eval += ne
        hist.append(fn)
        if st >= 0:
            return SQPResult(x, lam, st, k, fn, f0, n_eval, hist)
        if opts.stall_ratio > 0.0 and tol < fn <= opts.stall_tol * f0 and fn > opts.stall_ratio * fn_old:
            return SQPResult(x, lam, STALLED, k + 1, fn, f0, n_eval, hist)
    status = CONVERGED if fn <= tol else MAX_ITER
    return SQPResult(x, lam, status, opts.max_iter, fn, f0, n_eval, hist)


def sqp_solve_warm(model: ROMModel, mu, xhat0: np.ndarray, lam0: np.ndarray, opts: SQPOptions = SQPOptions()):
    """SQP warm-started from a proposal (xhat0, lam0), with the zero start as fallback: the
    zero start's first KKT residual norm f_zero (zero latents, least-squares multiplier) is
    computed first; the proposal is used only if its own first norm is finite and not larger.
    Tolerances are relative to f_zero either way.  Returns (result, used_fallback, f_zero,
    f_proposal)."""
    from .proposal import use_zero_start
    x_z = np.zeros(model.n_D)
    ev_z = evaluate(model, mu, x_z)
    lam_z, _ = start_multiplier(model, ev_z)
    f_zero = float(np.linalg.norm(kkt_rhs(model, ev_z, lam_z)))
    ev_p = evaluate(model, mu, np.asarray(xhat0, dtype=np.float64))
    f_prop = float(np.linalg.norm(kkt_rhs(model, ev_p, np.asarray(lam0, dtype=np.float64))))
    fb = use_zero_start(f_prop, f_zero)
    if fb:
        res = sqp_solve(model, mu, x_z, lam_z, opts, f_ref=f_zero)
    else:
        res = sqp_solve(model, mu, xhat0, lam0, opts, f_ref=f_zero)
    return res, fb, f_zero, f_prop


# ----------------------------------------------------------------------------------
# Post-solve metric (eq. relative_error)
# ----------------------------------------------------------------------------------

def relative_error(model: ROMModel, xhat: np.ndarray, x_fom: np.ndarray) -> float:
    tot = 0.0
    for i, (xo, xg) in enumerate(model.split(xhat)):
        sd = model.dd.subdomains[i]
        to, tg = x_fom[sd.omega], x_fom[sd.gamma]
        num = np.sum((to - _decode(model.dec_om[i], xo)) ** 2) + np.sum((tg - _decode(model.dec_ga[i], xg)) ** 2)
        tot += num / (np.sum(to ** 2) + np.sum(tg ** 2))
    return float(np.sqrt(tot / model.n_sub))


def relative_error_states(dd: DDMaps, states: list, x_fom: np.ndarray) -> float:
    """eq. relative_error for given subdomain states [(x^Omega, x^Gamma)]."""
    tot = 0.0
    for sd, (go, gg) in zip(dd.subdomains, states):
        to, tg = x_fom[sd.omega], x_fom[sd.gamma]
        tot += (np.sum((to - go) ** 2) + np.sum((tg - gg) ** 2)) / (np.sum(to ** 2) + np.sum(tg ** 2))
    return float(np.sqrt(tot / len(dd.subdomains)))


# ----------------------------------------------------------------------------------
# DD FOM through the same SQP (B_i = I, g = identity, constraints sum_i A_i x_i^Gamma = 0)
# ----------------------------------------------------------------------------------

def dd_fom_sqp(fom: BurgersFOM, dd: DDMaps, mu, x0_states=None, tol=1e-9, max_iter=50):
    """eq. fom_dd_nlp solved by Lagrange-Gauss-Newton SQP with full steps (Theorem 1
    setting).  Returns per-subdomain states, multiplier and the KKT residual history."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    subs = dd.subdomains
    sizes = [(len(s.omega), len(s.gamma)) for s in subs]
    offs = np.cumsum([0] + [a + b for a, b in sizes])
    nD, nA = int(offs[-1]), dd.n_A
    x = np.zeros(nD)
    if x0_states is not None:
        x = np.concatenate([np.concatenate(p) for p in x0_states])
    lam = np.zeros(nA)
    hist = []
    for it in range(max_iter + 1):
        blocks, rhs, Ecols = [], [], []
        c = np.zeros(nA)
        for i, (a, b) in enumerate(sizes):
            xo, xg = x[offs[i]:offs[i] + a], x[offs[i] + a:offs[i + 1]]
            r, dro, drg = subdomain_residual_jac(fom, dd, i, xo, xg, mu)
            R = sp.hstack([dro, drg]).tocsr()
            blocks.append((R.T @ R).tocsr())
            Ei = sp.hstack([sp.csr_matrix((nA, a)), dd.A[i]]).tocsr()
            Ecols.append(Ei)
            rhs.append(R.T @ r + Ei.T @ lam)
            c += dd.A[i] @ xg
        F = -np.concatenate(rhs + [c])
        hist.append(float(np.linalg.norm(F)))
        if hist[-1] <= tol or it == max_iter:
            break
        E = sp.hstack(Ecols).tocsr()
        K = sp.bmat([[sp.block_diag(blocks), E.T], [E, None]], format="csc")
        sol = spla.spsolve(K, F)
        x = x + sol[:nD]
        lam = lam + sol[nD:]
    states = [(x[offs[i]:offs[i] + a], x[offs[i] + a:offs[i + 1]]) for i, (a, b) in enumerate(sizes)]
    return states, lam, hist


def hr_interior_rows(model: ROMModel, i: int) -> np.ndarray:
    """Local indices (into x_i^Omega) of the interior DoFs that Z_i r_i reads: the u and v
    DoFs of the 5-point stencils of the sampled nodes that are interior states of
    subdomain i (Section 5.3: only these decoder outputs are needed)."""
    sd = model.dd.subdomains[i]
    g = model.grid
    n = g.n_nodes
    need = set()
    for q in np.asarray(model.hr_nodes[i]):
        j, ii = divmod(int(q), g.nx)
        for di, dj in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
            a, c = ii + di, j + dj
            if 0 <= a < g.nx and 0 <= c < g.ny:
                node = c * g.nx + a
                need.add(node)
                need.add(node + n)
    dofs = np.array(sorted(need), dtype=np.int64)
    pos = np.searchsorted(sd.omega, dofs)
    ok = (pos < len(sd.omega)) & (sd.omega[np.minimum(pos, len(sd.omega) - 1)] == dofs)
    return pos[ok]
