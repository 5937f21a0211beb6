"""Pins of the Burgers FOM oracle against what the paper and mathematics fix."""
import numpy as np
import pytest

from oracle.burgers import BurgersFOM, Grid, newton_fom, psi, u_exact, v_exact


def test_exact_solution_solves_pde():
    """u_ex, v_ex (eq. burgers_pde_exact_solution) satisfy the PDE: check the continuous
    residual with high-order finite differences at random points."""
    rng = np.random.default_rng(0)
    nu = 0.1
    for a, lam in [(1.0, 5.0), (100.0, 12.0), (1e4, 20.0)]:
        for _ in range(5):
            x, y = rng.uniform(-0.9, 0.9), rng.uniform(0.005, 0.045)
            h = 1e-3
            def d(f, dx, dy):
                return (-f(x + 2 * dx, y + 2 * dy) + 8 * f(x + dx, y + dy) - 8 * f(x - dx, y - dy) + f(x - 2 * dx, y - 2 * dy)) / (12 * h)
            def d2(f, dx, dy):
                return (-f(x + 2 * dx, y + 2 * dy) + 16 * f(x + dx, y + dy) - 30 * f(x, y) + 16 * f(x - dx, y - dy) - f(x - 2 * dx, y - 2 * dy)) / (12 * h * h)
            U = lambda X, Y: u_exact(X, Y, a, lam, nu)
            V = lambda X, Y: v_exact(X, Y, a, lam, nu)
            for F in (U, V):
                lhs = U(x, y) * d(F, h, 0) + V(x, y) * d(F, 0, h)
                rhs = nu * (d2(F, h, 0) + d2(F, 0, h))
                scale = abs(U(x, y) * d(F, h, 0)) + abs(nu * d2(F, 0, h)) + 1.0
                assert abs(lhs - rhs) / scale < 1e-5


def test_psi_positive_on_paper_domain():
    """Reading of the domain: psi > 0 on [-1,1]x[0,0.05] over the parameter box, but it
    changes sign on [-1,1]^2 (so the Dirichlet data would be singular there)."""
    X, Y = np.meshgrid(np.linspace(-1, 1, 201), np.linspace(0, 0.05, 51))
    for a in (1.0, 1e4):
        for lam in (5.0, 20.0):
            assert psi(X, Y, a, lam).min() > 0
    X2, Y2 = np.meshgrid(np.linspace(-1, 1, 201), np.linspace(-1, 1, 201))
    assert psi(X2, Y2, 1.0, 5.0).min() < 0


def test_second_order_convergence():
    """Discrete solution error against u_ex falls ~4x per halving of h (central FD)."""
    mu = (100.0, 5.0)
    errs = []
    for n in (10, 20, 40):
        f = BurgersFOM(Grid(n, n))
        res = newton_fom(f, mu)
        assert res.converged
        xe = f.exact_state(mu)
        errs.append(np.max(np.abs(res.x - xe)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # nested grids: h = 2/(n+1) does not halve exactly; compare against the h ratio
    hs = np.array([2.0 / (n + 1) for n in (10, 20, 40)])
    expected = 2 * np.log2(hs[:-1] / hs[1:])
    assert np.all(np.abs(rates - expected) < 0.15), (rates, expected)


def test_truncation_error_second_order():
    """r_h(u_ex) = O(h^2) (consistency of eq. burgers_discretized)."""
    mu = (50.0, 8.0)
    vals = []
    for n in (16, 32, 64):
        f = BurgersFOM(Grid(n, n))
        vals.append(np.max(np.abs(f.residual(f.exact_state(mu), mu))))
    r1 = np.log2(vals[0] / vals[1])
    r2 = np.log2(vals[1] / vals[2])
    assert 1.7 < r1 < 2.3 and 1.8 < r2 < 2.2, (vals, r1, r2)


def test_jacobian_central_differences():
    g = Grid(7, 5)
    f = BurgersFOM(g)
    mu = (300.0, 11.0)
    rng = np.random.default_rng(1)
    x = f.exact_state(mu) + 0.1 * rng.standard_normal(g.n_dof)
    J = f.jacobian(x, mu).toarray()
    Jfd = np.zeros_like(J)
    for k in range(g.n_dof):
        e = np.zeros(g.n_dof)
        h = 1e-6 * max(1.0, abs(x[k]))
        e[k] = h
        Jfd[:, k] = (f.residual(x + e, mu) - f.residual(x - e, mu)) / (2 * h)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))
    # six nonzeros per row away from the boundary (5-point stencil + the other field's centre)
    nnz = (np.abs(J) > 0).sum(1)
    assert nnz.max() == 6


def test_pointwise_stencil_form():
    """The Kronecker form equals the pointwise form -u D_x u - v D_y u + nu Lap_h u at an
    interior node (independent restatement of the discretisation)."""
    g = Grid(6, 5)
    f = BurgersFOM(g)
    mu = (20.0, 7.0)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.n_dof)
    r = f.residual(x, mu)
    n = g.n_nodes
    u = x[:n].reshape(g.ny, g.nx)
    v = x[n:].reshape(g.ny, g.nx)
    j, i = 2, 3
    Dx = lambda F: (F[j, i + 1] - F[j, i - 1]) / (2 * g.hx)
    Dy = lambda F: (F[j + 1, i] - F[j - 1, i]) / (2 * g.hy)
    L = lambda F: (F[j, i + 1] - 2 * F[j, i] + F[j, i - 1]) / g.hx ** 2 + (F[j + 1, i] - 2 * F[j, i] + F[j - 1, i]) / g.hy ** 2
    ru = -u[j, i] * Dx(u) - v[j, i] * Dy(u) + g.nu * L(u)
    rv = -u[j, i] * Dx(v) - v[j, i] * Dy(v) + g.nu * L(v)
    k = j * g.nx + i
    assert np.isclose(r[k], ru, rtol=1e-12, atol=1e-9)
    assert np.isclose(r[n + k], rv, rtol=1e-12, atol=1e-9)
