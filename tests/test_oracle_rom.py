"""Pins of the SQP oracle: Theorem 1, Lemma 2, KKT conditions at convergence, the
single-domain Gauss-Newton special case, the identity-activation LS-ROM special case
(against an independently written LS-ROM solver, itself pinned by Theorem 1), central
differences of the per-subdomain Jacobians, the initial multiplier, the stagnation stop
and the relative-error metric."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.autoencoder import ACT_IDENTITY, ACT_SIGMOID, ACT_SWISH, Decoder
from oracle.burgers import BurgersFOM, Grid, newton_fom
from oracle.ddmaps import build_dd, restrict
from oracle.pack import load_pack
from oracle import lsrom
from oracle.rom import (CONVERGED, LINESEARCH_FAIL, MAX_ITER, STALLED, ROMModel, SQPOptions, dd_fom_sqp, evaluate,
                        initial_multiplier, kkt_rhs, kkt_step, relative_error_states, sqp_solve, sqp_step)


def test_theorem1_dd_fom_equals_monolithic():
    """The DD-FOM (B = I, g = id, constraints sum A_i x_i^Gamma = 0) solved by the SQP
    method gives the monolithic Newton solution restricted to the subdomains."""
    g = Grid(12, 8)
    f = BurgersFOM(g)
    mu = (2500.0, 14.0)
    xm = newton_fom(f, mu).x
    for sx, sy in ((2, 2), (3, 2)):
        dd = build_dd(g, sx, sy)
        states, lam, hist = dd_fom_sqp(f, dd, mu, tol=1e-9 * 1e6)
        for (xo, xg), (to, tg) in zip(states, restrict(dd, xm)):
            assert np.linalg.norm(xo - to) <= 1e-10 * np.linalg.norm(to)
            assert np.linalg.norm(xg - tg) <= 1e-10 * np.linalg.norm(tg)
        assert relative_error_states(dd, states, xm) < 1e-10


def _affine_decoder(N, n, b, s, x0, rng, activation):
    w = N * s
    W1 = 0.5 * rng.standard_normal((w, n))
    b1 = 0.1 * rng.standard_normal(w)
    W2 = 0.01 * rng.standard_normal((N, 3, b))
    return Decoder(W1, b1, W2, x0.copy(), b, s, activation)


def _random_model(activation=ACT_SIGMOID, seed=0, hr=True, nsx=2, nsy=2, mu0=(800.0, 9.0)):
    g = Grid(12, 8)
    f = BurgersFOM(g)
    dd = build_dd(g, nsx, nsy)
    xs = newton_fom(f, mu0).x
    rng = np.random.default_rng(seed)
    dec_om, dec_ga, hr_nodes = [], [], []
    for sd in dd.subdomains:
        dec_om.append(_affine_decoder(len(sd.omega), 3, 3, 2, xs[sd.omega], rng, activation))
        n_ga = 2 if len(sd.gamma) else 0
        dec_ga.append(_affine_decoder(len(sd.gamma), n_ga, 3, 2, xs[sd.gamma], rng, activation))
        hr_nodes.append(np.sort(rng.choice(sd.own_nodes, size=max(4, len(sd.own_nodes) // 2), replace=False)))
    n_C = sum(d.n for d in dec_ga) // 2
    C = si.gaussian_matrix(n_C, dd.n_A, seed + 100)
    return ROMModel(g, nsx, nsy, dec_om, dec_ga, hr_nodes if hr else None, C, dd=dd, fom=f)


def test_lemma2_step_solves_qp():
    """The KKT step equals the minimiser of the QP (eq. dd_lspg_NLP_general_QP), computed
    independently by a null-space method."""
    m = _random_model()
    mu = (1200.0, 10.0)
    x = 0.3 * np.random.default_rng(1).standard_normal(m.n_D)
    ev = evaluate(m, mu, x)
    lam = np.random.default_rng(2).standard_normal(m.n_C)
    sx, sl = kkt_step(m, ev, lam)
    # QP: min 0.5 sum ||Zr_i + ZR_i s_i||^2  s.t.  c + E s = 0
    nD = m.n_D
    E = np.zeros((m.n_C, nD))
    ZR = np.zeros((sum(z.shape[0] for z in ev.ZR), nD))
    Zr = np.concatenate(ev.Zr)
    r0 = 0
    for i, (o, (a, b)) in enumerate(zip(m.offsets(), m.sizes())):
        E[:, o + a:o + a + b] = ev.EG[i]
        ZR[r0:r0 + ev.ZR[i].shape[0], o:o + a + b] = ev.ZR[i]
        r0 += ev.ZR[i].shape[0]
    sp_ = np.linalg.lstsq(E, -ev.c, rcond=None)[0]
    _, _, Vt = np.linalg.svd(E)
    Nz = Vt[m.n_C:].T
    y = np.linalg.lstsq(ZR @ Nz, -(Zr + ZR @ sp_), rcond=None)[0]
    s_qp = sp_ + Nz @ y
    assert np.linalg.norm(sx - s_qp) <= 1e-9 * np.linalg.norm(s_qp)
    # the QP multiplier is lambda + s_lambda
    lam_qp = np.linalg.lstsq(E.T, -(ZR.T @ (Zr + ZR @ s_qp)), rcond=None)[0]
    assert np.linalg.norm(lam + sl - lam_qp) <= 1e-7 * max(1.0, np.linalg.norm(lam_qp))


def test_kkt_conditions_at_convergence(tiny_pack):
    m = load_pack(tiny_pack)
    mu = si.heldout_mu(1, 11)[0]
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-10))
    assert res.status == CONVERGED
    ev = evaluate(m, mu, res.xhat)
    F = kkt_rhs(m, ev, res.lam)
    nD = m.n_D
    assert np.linalg.norm(F[:nD]) <= 1e-9 * res.fnorm0        # stationarity
    assert np.linalg.norm(F[nD:]) <= 1e-9 * res.fnorm0        # feasibility of the weak constraint


def test_single_domain_is_gauss_newton():
    """With one subdomain there is no constraint and the SQP iteration is Gauss-Newton on
    min ||Z r(g(xhat))|| (the single-domain case of Section 7.5): its limit equals that of a
    plain Gauss-Newton loop on fourth-order central-difference Jacobians of the residual
    (nothing of evaluate()'s chain rule enters)."""
    m = _random_model(nsx=1, nsy=1, seed=3)
    mu = (900.0, 9.5)
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=200, tol_abs=0.0, tol_rel=1e-13))
    assert res.status == CONVERGED, res.status

    def fun(x):
        return evaluate(m, mu, x).Zr[0]

    def jac(x, h=1e-3):
        cols = []
        for k in range(m.n_D):
            e = np.zeros(m.n_D)
            e[k] = h
            cols.append((-fun(x + 2 * e) + 8 * fun(x + e) - 8 * fun(x - e) + fun(x - 2 * e)) / (12 * h))
        return np.stack(cols, axis=1)

    x = np.zeros(m.n_D)
    for _ in range(80):
        x = x - np.linalg.lstsq(jac(x), fun(x), rcond=None)[0]
    assert np.linalg.norm(res.xhat - x) <= 1e-9 * max(1.0, np.linalg.norm(x))


def _affine_maps(m):
    """sigma = id: g(xhat) = (x_ref + W2 b1) + (W2 W1) xhat for every decoder of m."""
    om = [(d.x_ref + d.W2() @ d.b1, np.asarray(d.W2() @ d.W1)) for d in m.dec_om]
    ga = [(d.x_ref + d.W2() @ d.b1, np.asarray(d.W2() @ d.W1)) for d in m.dec_ga]
    return om, ga


def test_lsrom_full_basis_is_dd_fom():
    """The independent LS-ROM solver with identity bases (Phi_i = I), B_i = I and C = I is the
    DD FOM (eq. fom_dd_nlp): by Theorem 1 its solution is the monolithic Newton solution
    restricted to the subdomains.  This pins the LS-ROM solver (prolongation, QP step,
    multipliers, line search) against a different algorithm."""
    g = Grid(12, 8)
    f = BurgersFOM(g)
    dd = build_dd(g, 2, 2)
    mu = (1800.0, 12.0)
    xm = newton_fom(f, mu).x
    eye = lambda N: np.eye(N)
    rom = lsrom.LSROM(f, dd, np.eye(dd.n_A), [np.zeros(len(sd.omega)) for sd in dd.subdomains],
                      [eye(len(sd.omega)) for sd in dd.subdomains], [np.zeros(len(sd.gamma)) for sd in dd.subdomains],
                      [eye(len(sd.gamma)) for sd in dd.subdomains], hr=None)
    res = lsrom.solve(rom, mu, max_iter=60, tol_abs=0.0, tol_rel=1e-12)
    assert res.status == lsrom.CONVERGED, res.status
    o = 0
    for sd in dd.subdomains:
        a, b = len(sd.omega), len(sd.gamma)
        assert np.linalg.norm(res.xhat[o:o + a] - xm[sd.omega]) <= 1e-10 * np.linalg.norm(xm[sd.omega])
        assert np.linalg.norm(res.xhat[o + a:o + a + b] - xm[sd.gamma]) <= 1e-10 * np.linalg.norm(xm[sd.gamma])
        o += a + b


def test_identity_activation_equals_lsrom():
    """sigma = id makes g affine: g(xhat) = (x_ref + W2 b1) + (W2 W1) xhat (Sections 3.3, 3.4).
    The NM-ROM SQP of rom.py then equals the independent LS-ROM solver (its own residual
    Jacobian route, null-space QP steps, Cholesky initial multiplier) iterate for iterate."""
    m = _random_model(activation=ACT_IDENTITY, seed=5)
    mu = (1000.0, 9.2)
    for max_iter in (1, 2, 40):
        opts = SQPOptions(max_iter=max_iter, tol_abs=0.0, tol_rel=1e-12)
        res = sqp_solve(m, mu, opts=opts)
        om, ga = _affine_maps(m)
        rom = lsrom.LSROM(m.fom, m.dd, m.C, [a for a, _ in om], [b for _, b in om], [a for a, _ in ga],
                          [b for _, b in ga], hr=[lsrom.collocation_operator(m.grid, q) for q in m.hr_nodes])
        res2 = lsrom.solve(rom, mu, max_iter=max_iter, tol_abs=0.0, tol_rel=1e-12)
        assert res.status == res2.status and res.iters == res2.iters, (max_iter, res.status, res2.status)
        assert np.linalg.norm(res.xhat - res2.xhat) <= 1e-10 * max(1.0, np.linalg.norm(res2.xhat))
        assert np.linalg.norm(res.lam - res2.lam) <= 1e-8 * max(1.0, np.linalg.norm(res2.lam))
        assert abs(res.fnorm0 - res2.fnorm0) <= 1e-10 * res2.fnorm0
    assert res.status == CONVERGED


@pytest.mark.parametrize("activation", [ACT_SIGMOID, ACT_SWISH, ACT_IDENTITY])
def test_evaluate_derivatives_central_differences(activation):
    """Z R_i = d(Z r_i)/dxhat and E_i = dc/dxhat_i^Gamma (eq. gauss_newton_hessian,
    eq. optimality_residuals), checked by central differences over the whole latent vector:
    each block sits at its own subdomain's columns (interior, then interface) and the other
    columns vanish.  The KKT right-hand side is minus the gradient of the Lagrangian."""
    m = _random_model(activation=activation, seed=11)
    mu = (1500.0, 11.0)
    rng = np.random.default_rng(3)
    x = 0.4 * rng.standard_normal(m.n_D)
    lam = rng.standard_normal(m.n_C)
    ev = evaluate(m, mu, x)
    h = 1e-6
    dZr = [np.zeros((z.shape[0], m.n_D)) for z in ev.Zr]
    dc = np.zeros((m.n_C, m.n_D))
    dL = np.zeros(m.n_D)

    def lagrangian(e):
        return 0.5 * sum(float(z @ z) for z in e.Zr) + float(lam @ e.c)

    for k in range(m.n_D):
        e = np.zeros(m.n_D)
        e[k] = h
        ep, em = evaluate(m, mu, x + e), evaluate(m, mu, x - e)
        for i in range(m.n_sub):
            dZr[i][:, k] = (ep.Zr[i] - em.Zr[i]) / (2 * h)
        dc[:, k] = (ep.c - em.c) / (2 * h)
        dL[k] = (lagrangian(ep) - lagrangian(em)) / (2 * h)
    Efull = np.zeros((m.n_C, m.n_D))
    for i, (o, (a, b)) in enumerate(zip(m.offsets(), m.sizes())):
        ref = np.zeros_like(dZr[i])
        ref[:, o:o + a + b] = ev.ZR[i]
        assert np.max(np.abs(dZr[i] - ref)) <= 1e-6 * max(1.0, np.max(np.abs(ref)))
        Efull[:, o + a:o + a + b] = ev.EG[i]
    assert np.max(np.abs(dc - Efull)) <= 1e-7 * max(1.0, np.max(np.abs(Efull)))
    F = kkt_rhs(m, ev, lam)
    assert np.max(np.abs(-F[:m.n_D] - dL)) <= 1e-6 * max(1.0, np.max(np.abs(dL)))
    assert np.array_equal(-F[m.n_D:], ev.c)


def test_initial_multiplier_least_squares():
    """lambda^0 = argmin ||grad_xhat f + (dc/dxhat)^T lambda|| (the first-order conditions in
    the latents, with f the HR objective): its residual is orthogonal to the range of the
    constraint Jacobian's transpose, and perturbing it only grows the residual.  The
    gradient and the constraint Jacobian are taken by central differences, not from
    evaluate()."""
    m = _random_model(seed=13)
    mu = (700.0, 8.0)
    x = 0.3 * np.random.default_rng(4).standard_normal(m.n_D)
    ev = evaluate(m, mu, x)
    lam0 = initial_multiplier(m, ev)
    h = 1e-6
    grad = np.zeros(m.n_D)
    E = np.zeros((m.n_C, m.n_D))
    for k in range(m.n_D):
        e = np.zeros(m.n_D)
        e[k] = h
        ep, em = evaluate(m, mu, x + e), evaluate(m, mu, x - e)
        grad[k] = (0.5 * sum(float(z @ z) for z in ep.Zr) - 0.5 * sum(float(z @ z) for z in em.Zr)) / (2 * h)
        E[:, k] = (ep.c - em.c) / (2 * h)
    res = grad + E.T @ lam0
    assert np.linalg.norm(E @ res) <= 1e-6 * np.linalg.norm(E) * np.linalg.norm(grad)
    rng = np.random.default_rng(5)
    base = np.linalg.norm(res)
    for _ in range(5):
        d = 1e-3 * rng.standard_normal(m.n_C) * max(1.0, np.linalg.norm(lam0))
        assert np.linalg.norm(grad + E.T @ (lam0 + d)) > base


def test_stall_rule(tiny_pack):
    """Stagnation stop (reading of the stopping rule for reduced-precision decoders): with an
    unreachable tolerance, FP64 SQP runs until rounding stops the Armijo test from passing.
    With stall_tol set, the solve then ends STALLED at a point whose ||F|| is below
    stall_tol ||F_0||, where the full step indeed fails the Armijo test; with stall_tol = 0
    the same solve ends LINESEARCH_FAIL or MAX_ITER instead, and a stall_tol below the
    reached ||F|| / ||F_0|| never reports STALLED."""
    m = load_pack(tiny_pack)
    mu = si.heldout_mu(1, 11)[0]
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=200, tol_abs=0.0, tol_rel=0.0, stall_tol=1e-6))
    assert res.status == STALLED, res.status
    assert res.fnorm <= 1e-6 * res.fnorm0
    ev = evaluate(m, mu, res.xhat)
    sx, sl = kkt_step(m, ev, res.lam)
    F0 = kkt_rhs(m, ev, res.lam)
    F1 = kkt_rhs(m, evaluate(m, mu, res.xhat + sx), res.lam + sl)
    assert 0.5 * float(F1 @ F1) > (1.0 - 2.0 * 1e-4) * 0.5 * float(F0 @ F0)
    res0 = sqp_solve(m, mu, opts=SQPOptions(max_iter=res.iters + 3, tol_abs=0.0, tol_rel=0.0, stall_tol=0.0))
    assert res0.status in (LINESEARCH_FAIL, MAX_ITER)
    tight = 0.5 * res.fnorm / res.fnorm0
    r2 = sqp_solve(m, mu, opts=SQPOptions(max_iter=res.iters, tol_abs=0.0, tol_rel=0.0, stall_tol=tight * 1e-3))
    assert r2.status != STALLED


def test_relative_error_zero_for_exact_states():
    m = _random_model(seed=7)
    x = newton_fom(m.fom, (800.0, 9.0)).x
    states = restrict(m.dd, x)
    assert relative_error_states(m.dd, states, x) == 0.0
    # and positive for a perturbed state, with the eq. relative_error scaling
    pert = [(a * 1.01, b * 1.01) for a, b in states]
    assert np.isclose(relative_error_states(m.dd, pert, x), 0.01, rtol=1e-12)


def test_cfg0_solve_converges(cfg0_pack):
    """The 36x36 workload: zero-start SQP reaches the relative KKT tolerance."""
    m = load_pack(cfg0_pack)
    mu = si.heldout_mu(1, 0)[0]
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=50, tol_abs=0.0, tol_rel=1e-8))
    assert res.status == CONVERGED
    assert res.fnorm <= 1e-8 * res.fnorm0


# ---- stop statuses (Lemma 1 hypotheses, non-finite data, line search, iteration cap) ----

def test_rank_deficient_constraint_stops_kkt_not_pd(tiny_pack):
    """A zero row of C gives the constraint Jacobian a zero row: the KKT matrix of
    eq. sqp_system has an exactly zero row (it is singular, Lemma 1's full-row-rank
    hypothesis fails) and the least-squares multiplier is not unique.  The solve stops at
    once with KKT_NOT_PD, lambda = 0, at the start point."""
    from oracle.rom import KKT_NOT_PD, constraint_full_row_rank, kkt_matrix
    from status_cases import rank_deficient_constraint
    m = load_pack(rank_deficient_constraint(tiny_pack))
    mu = si.heldout_mu(1, 11)[0]
    ev = evaluate(m, mu, np.zeros(m.n_D))
    K = kkt_matrix(m, ev)
    assert np.all(K[m.n_D] == 0.0)
    assert not constraint_full_row_rank(m, ev)
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=20, tol_abs=0.0, tol_rel=1e-10))
    assert res.status == KKT_NOT_PD and res.iters == 0
    assert np.all(res.xhat == 0.0) and np.all(res.lam == 0.0)
    assert res.fnorm == np.linalg.norm(kkt_rhs(m, ev, np.zeros(m.n_C)))


def test_singular_block_stops_kkt_not_pd(tiny_pack):
    """A zero column of an interior decoder's W1 makes Z R_0 lose a column exactly, so H_0
    (and the KKT matrix) has a zero row: Lemma 1's positive-definiteness hypothesis fails at
    the first step.  The solve stops with KKT_NOT_PD at the start point with the
    least-squares multiplier."""
    from oracle.rom import KKT_NOT_PD, kkt_matrix
    from status_cases import singular_block
    m = load_pack(singular_block(tiny_pack, sd=0, col=1))
    mu = si.heldout_mu(1, 11)[0]
    ev = evaluate(m, mu, np.zeros(m.n_D))
    assert np.all(ev.H[0][1] == 0.0) and np.all(kkt_matrix(m, ev)[1] == 0.0)
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=20, tol_abs=0.0, tol_rel=1e-10))
    assert res.status == KKT_NOT_PD and res.iters == 0
    assert np.all(res.xhat == 0.0)
    assert np.allclose(res.lam, initial_multiplier(m, ev), rtol=0, atol=0)


def test_nonfinite_parameter_stops_nonfinite(tiny_pack):
    """A NaN parameter makes the Dirichlet data, hence the first KKT residual, NaN."""
    from oracle.rom import NONFINITE
    m = load_pack(tiny_pack)
    for mu in ((np.nan, 10.0), (500.0, np.nan)):
        res = sqp_solve(m, mu, opts=SQPOptions(max_iter=10))
        assert res.status == NONFINITE and res.iters == 0 and not np.isfinite(res.fnorm)


def test_linesearch_fail_without_backtracking(tiny_pack):
    """max_backtracks = 0: the solve stops with LINESEARCH_FAIL exactly where the full KKT step
    fails the Armijo test phi(1) <= (1 - 2 c1) phi(0), recomputed here from the returned point."""
    m = load_pack(tiny_pack)
    mus = si.heldout_mu(8, 17)
    seen = 0
    for mu in mus:
        res = sqp_solve(m, mu, opts=SQPOptions(max_iter=10, tol_abs=0.0, tol_rel=1e-12, max_backtracks=0))
        if res.status != LINESEARCH_FAIL:
            continue
        seen += 1
        ev = evaluate(m, mu, res.xhat)
        sx, sl = kkt_step(m, ev, res.lam)
        F0 = kkt_rhs(m, ev, res.lam)
        F1 = kkt_rhs(m, evaluate(m, mu, res.xhat + sx), res.lam + sl)
        assert 0.5 * float(F1 @ F1) > (1.0 - 2.0 * 1e-4) * 0.5 * float(F0 @ F0)
        assert res.fnorm == np.linalg.norm(F0)
    assert seen >= 2


def test_max_iter_one_is_one_step(tiny_pack):
    """max_iter = 1 stops after one accepted step (MAX_ITER unless it already converged) at the
    point sqp_step returns from the start."""
    from oracle.rom import start_multiplier
    m = load_pack(tiny_pack)
    for mu in si.heldout_mu(3, 19):
        res = sqp_solve(m, mu, opts=SQPOptions(max_iter=1, tol_abs=0.0, tol_rel=1e-12))
        x0 = np.zeros(m.n_D)
        ev = evaluate(m, mu, x0)
        lam0, ok = start_multiplier(m, ev)
        assert ok
        x1, l1, _, f1, st, _, _ = sqp_step(m, mu, x0, lam0, SQPOptions(), ev)
        assert st == -1 and res.status == MAX_ITER and res.iters == 1
        assert np.array_equal(res.xhat, x1) and np.array_equal(res.lam, l1) and res.fnorm == f1


def test_stall_ratio_rule(tiny_pack):
    """The progress form of the stagnation stop: with stall_ratio > 0 the solve stops STALLED at
    the first accepted step that ends below stall_tol ||F_0|| (above the tolerance) having reduced
    ||F|| by less than the factor stall_ratio - read off the history of the same solve run
    without the rule, whose iterate at that step it returns exactly."""
    m = load_pack(tiny_pack)
    for mu in si.heldout_mu(3, 11):
        free = sqp_solve(m, mu, opts=SQPOptions(max_iter=60, tol_abs=0.0, tol_rel=1e-14))
        h = free.hist if hasattr(free, "hist") else free.history
        theta, st = 0.05, 1e-3
        k_stop = next((k for k in range(1, len(h)) if h[k] <= st * free.fnorm0 and h[k] > theta * h[k - 1]), None)
        assert k_stop is not None
        res = sqp_solve(m, mu, opts=SQPOptions(max_iter=60, tol_abs=0.0, tol_rel=1e-14, stall_tol=st,
                                               stall_ratio=theta))
        assert res.status == STALLED and res.iters == k_stop
        ref = sqp_solve(m, mu, opts=SQPOptions(max_iter=k_stop, tol_abs=0.0, tol_rel=1e-14))
        assert np.array_equal(res.xhat, ref.xhat) and res.fnorm == h[k_stop]
