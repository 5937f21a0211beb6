"""Pins of the SQP oracle: Theorem 1, Lemma 2, KKT conditions at convergence, the
single-domain Gauss-Newton special case, the identity-activation LS-ROM special case and
the relative-error metric."""
import numpy as np
import pytest
import scipy.optimize as so

import seeded_inputs as si
from oracle.autoencoder import ACT_IDENTITY, ACT_SIGMOID, Decoder, decode
from oracle.burgers import BurgersFOM, Grid, newton_fom
from oracle.ddmaps import build_dd, restrict
from oracle.pack import load_pack
from oracle.rom import (CONVERGED, AffineMap, ROMModel, SQPOptions, dd_fom_sqp, evaluate, kkt_rhs, kkt_step,
                        lsrom_decoders, relative_error, relative_error_states, sqp_solve, sqp_solve_with)


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
    min ||Z r(g(xhat))||: its limit equals scipy's least-squares minimiser."""
    m = _random_model(nsx=1, nsy=1, seed=3)
    mu = (900.0, 9.5)
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=80, tol_abs=0.0, tol_rel=1e-11))
    assert res.status == CONVERGED, res.status

    def fun(x):
        return evaluate(m, mu, x).Zr[0]

    def jac(x):
        return evaluate(m, mu, x).ZR[0]

    ls = so.least_squares(fun, np.zeros(m.n_D), jac=jac, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15)
    assert np.linalg.norm(res.xhat - ls.x) <= 1e-7 * max(1.0, np.linalg.norm(ls.x))


def test_identity_activation_equals_lsrom():
    """sigma = id makes g affine: g(xhat) = (x_ref + W2 b1) + (W2 W1) xhat.  The NM-ROM SQP
    equals the SQP run with the explicit affine (LS-ROM) maps."""
    m = _random_model(activation=ACT_IDENTITY, seed=5)
    mu = (1000.0, 9.2)
    opts = SQPOptions(max_iter=40, tol_abs=0.0, tol_rel=1e-12)
    res = sqp_solve(m, mu, opts=opts)
    maps_om = [AffineMap(d.x_ref + d.W2() @ d.b1, d.W2() @ d.W1) for d in m.dec_om]
    maps_ga = [AffineMap(d.x_ref + d.W2() @ d.b1, d.W2() @ d.W1) for d in m.dec_ga]
    res2 = sqp_solve_with(m, mu, lsrom_decoders(maps_om, maps_ga), np.zeros(m.n_D), opts)
    assert res.status == CONVERGED and res2.status == CONVERGED
    assert np.linalg.norm(res.xhat - res2.xhat) <= 1e-10 * max(1.0, np.linalg.norm(res2.xhat))
    assert res.iters == res2.iters


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
