"""2D steady viscous Burgers FOM (Section 7.1), FP64, in the paper's matrix form.

Exact solution (eq. burgers_pde_exact_solution): u_ex, v_ex built from psi; its
boundary restriction is the Dirichlet data.  Discretisation (eq. burgers_discretized):

    r_u = u o (B_x u - b_ux) + v o (B_y u - b_uy) + C u + c_u
    r_v = u o (B_x v - b_vx) + v o (B_y v - b_vy) + C v + c_v

with B_x = -(1/2h_x) I (x) Bt_x, B_y = -(1/2h_y) Bt_y (x) I,
C = nu/h_x^2 I (x) Ct_x + nu/h_y^2 Ct_y (x) I, and the boundary vectors b_*, c_*
assembled from u_ex, v_ex on the four sides.  u and v are stacked x-fastest and the
state is x = [u; v] (reading: the paper orders each field x-fastest and is silent on
how the two fields are combined).

Domain: [-1, 1] x [0, L_y] with L_y = 0.05 (reading: the paper's box; on [-1,1]^2 the
closed form's denominator psi changes sign, so the Dirichlet data would be singular).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

NU_DEFAULT = 0.1
LY_DEFAULT = 0.05


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nu: float = NU_DEFAULT
    ly: float = LY_DEFAULT

    @property
    def hx(self) -> float:
        return 2.0 / (self.nx + 1)

    @property
    def hy(self) -> float:
        return self.ly / (self.ny + 1)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny

    @property
    def n_dof(self) -> int:
        return 2 * self.nx * self.ny

    def x(self, i):
        return -1.0 + np.asarray(i) * self.hx

    def y(self, j):
        return np.asarray(j) * self.hy


def psi(x, y, a, lam):
    """psi(x, y; a, lambda) = a(1+x) + (e^{lam(x-1)} + e^{-lam(x-1)}) cos(lam y)."""
    return a * (1.0 + x) + (np.exp(lam * (x - 1.0)) + np.exp(-lam * (x - 1.0))) * np.cos(lam * y)


def u_exact(x, y, a, lam, nu=NU_DEFAULT):
    return -2.0 * nu * (a + lam * (np.exp(lam * (x - 1.0)) - np.exp(-lam * (x - 1.0))) * np.cos(lam * y)) / psi(x, y, a, lam)


def v_exact(x, y, a, lam, nu=NU_DEFAULT):
    return 2.0 * nu * (lam * (np.exp(lam * (x - 1.0)) + np.exp(-lam * (x - 1.0))) * np.sin(lam * y)) / psi(x, y, a, lam)


@dataclass
class Operators:
    """Constant matrices of eq. burgers_discretized for one grid."""
    Bx: sp.csr_matrix
    By: sp.csr_matrix
    C: sp.csr_matrix


def _tri(n, lo, di, up):
    return sp.diags([lo * np.ones(n - 1), di * np.ones(n), up * np.ones(n - 1)], [-1, 0, 1], format="csr")


def operators(g: Grid) -> Operators:
    Btx = _tri(g.nx, -1.0, 0.0, 1.0)
    Bty = _tri(g.ny, -1.0, 0.0, 1.0)
    Ctx = _tri(g.nx, 1.0, -2.0, 1.0)
    Cty = _tri(g.ny, 1.0, -2.0, 1.0)
    Ix = sp.identity(g.nx, format="csr")
    Iy = sp.identity(g.ny, format="csr")
    Bx = (-1.0 / (2.0 * g.hx)) * sp.kron(Iy, Btx, format="csr")
    By = (-1.0 / (2.0 * g.hy)) * sp.kron(Bty, Ix, format="csr")
    C = (g.nu / g.hx ** 2) * sp.kron(Iy, Ctx, format="csr") + (g.nu / g.hy ** 2) * sp.kron(Cty, Ix, format="csr")
    return Operators(Bx.tocsr(), By.tocsr(), C.tocsr())


@dataclass
class BoundaryVectors:
    bx_u: np.ndarray  # b_{u,x}
    by_u: np.ndarray
    c_u: np.ndarray
    bx_v: np.ndarray
    by_v: np.ndarray
    c_v: np.ndarray


def boundary_vectors(g: Grid, a: float, lam: float) -> BoundaryVectors:
    """b_{u,x}, b_{u,y}, c_u and the v counterparts (the b_{.yl}/b_{.yr} of the
    definition are read as the bottom/top vectors b_{.yb}/b_{.yt})."""
    nx, ny, nu = g.nx, g.ny, g.nu
    xs = g.x(np.arange(1, nx + 1))
    ys = g.y(np.arange(1, ny + 1))
    x0, xr = g.x(0), g.x(nx + 1)
    y0, yt = g.y(0), g.y(ny + 1)
    e_first_x = np.zeros(nx); e_first_x[0] = 1.0
    e_last_x = np.zeros(nx); e_last_x[-1] = 1.0
    e_first_y = np.zeros(ny); e_first_y[0] = 1.0
    e_last_y = np.zeros(ny); e_last_y[-1] = 1.0

    out = {}
    for name, f in (("u", u_exact), ("v", v_exact)):
        bxl = np.kron(f(x0, ys, a, lam, nu), e_first_x)
        bxr = np.kron(f(xr, ys, a, lam, nu), e_last_x)
        byb = np.kron(e_first_y, f(xs, y0, a, lam, nu))
        byt = np.kron(e_last_y, f(xs, yt, a, lam, nu))
        out["bx_" + name] = (-1.0 / (2.0 * g.hx)) * (bxl - bxr)
        out["by_" + name] = (-1.0 / (2.0 * g.hy)) * (byb - byt)
        out["c_" + name] = (nu / g.hx ** 2) * (bxl + bxr) + (nu / g.hy ** 2) * (byb + byt)
    return BoundaryVectors(**out)


class BurgersFOM:
    """Residual r(x; mu) and its sparse Jacobian for x = [u; v]."""

    def __init__(self, g: Grid):
        self.g = g
        self.ops = operators(g)
        self._bv_cache: dict = {}

    def bv(self, mu) -> BoundaryVectors:
        key = (float(mu[0]), float(mu[1]))
        if key not in self._bv_cache:
            if len(self._bv_cache) > 64:
                self._bv_cache.clear()
            self._bv_cache[key] = boundary_vectors(self.g, key[0], key[1])
        return self._bv_cache[key]

    def residual(self, x: np.ndarray, mu) -> np.ndarray:
        o, b = self.ops, self.bv(mu)
        n = self.g.n_nodes
        u, v = x[:n], x[n:]
        ru = u * (o.Bx @ u - b.bx_u) + v * (o.By @ u - b.by_u) + o.C @ u + b.c_u
        rv = u * (o.Bx @ v - b.bx_v) + v * (o.By @ v - b.by_v) + o.C @ v + b.c_v
        return np.concatenate([ru, rv])

    def jacobian(self, x: np.ndarray, mu) -> sp.csr_matrix:
        o, b = self.ops, self.bv(mu)
        n = self.g.n_nodes
        u, v = x[:n], x[n:]
        D = sp.diags
        duu = D(o.Bx @ u - b.bx_u) + D(u) @ o.Bx + D(v) @ o.By + o.C
        duv = D(o.By @ u - b.by_u)
        dvu = D(o.Bx @ v - b.bx_v)
        dvv = D(u) @ o.Bx + D(o.By @ v - b.by_v) + D(v) @ o.By + o.C
        return sp.bmat([[duu, duv], [dvu, dvv]], format="csr")

    def exact_state(self, mu) -> np.ndarray:
        """Exact solution sampled at the interior nodes, x = [u; v]."""
        g = self.g
        X, Y = np.meshgrid(g.x(np.arange(1, g.nx + 1)), g.y(np.arange(1, g.ny + 1)), indexing="xy")
        return np.concatenate([u_exact(X, Y, mu[0], mu[1], g.nu).ravel(), v_exact(X, Y, mu[0], mu[1], g.nu).ravel()])


@dataclass
class NewtonResult:
    x: np.ndarray
    converged: bool
    iters: int
    res_history: list = field(default_factory=list)   # residual vectors r(x^(k)), k = 0..iters
    norms: list = field(default_factory=list)


def newton_fom(fom: BurgersFOM, mu, x0: np.ndarray | None = None, rtol: float = 1e-12,
               max_iter: int = 50, keep_history: bool = False) -> NewtonResult:
    """Monolithic Newton on r(x; mu) = 0 with Armijo backtracking on ||r||_2.

    Reading (the paper gives neither start nor tolerance): start from the zero interior
    state; stop when ||r||_2 <= rtol * max(1, ||r(x0)||_2)."""
    x = np.zeros(fom.g.n_dof) if x0 is None else np.array(x0, dtype=np.float64)
    r = fom.residual(x, mu)
    n0 = np.linalg.norm(r)
    hist = [r.copy()] if keep_history else []
    norms = [n0]
    target = rtol * max(1.0, n0)
    for k in range(max_iter):
        nr = norms[-1]
        if nr <= target:
            return NewtonResult(x, True, k, hist, norms)
        J = fom.jacobian(x, mu)
        dx = spla.spsolve(J.tocsc(), -r)
        alpha = 1.0
        for _ in range(30):
            xt = x + alpha * dx
            rt = fom.residual(xt, mu)
            if np.linalg.norm(rt) <= (1.0 - 1e-4 * alpha) * nr:
                break
            alpha *= 0.5
        x, r = xt, rt
        norms.append(np.linalg.norm(r))
        if keep_history:
            hist.append(r.copy())
    return NewtonResult(x, norms[-1] <= target, max_iter, hist, norms)


def solve_fom(fom: BurgersFOM, mu, keep_history=False, rtol=1e-12) -> NewtonResult:
    """Newton from zero; if that fails, restart from the exact solution sampled on the grid."""
    res = newton_fom(fom, mu, None, rtol=rtol, keep_history=keep_history)
    if not res.converged:
        res2 = newton_fom(fom, mu, fom.exact_state(mu), rtol=rtol, keep_history=keep_history)
        if keep_history:
            res2.res_history = res.res_history + res2.res_history
        res = res2
    return res
