"""Pins of the DD maps, the masked autoencoder and HR against the paper's integers,
closed forms and finite differences."""
import numpy as np
import pytest

from oracle.autoencoder import (ACT_IDENTITY, ACT_SIGMOID, ACT_SWISH, Adam, MaskedAE, band_mask,
                                decode_jacobian, export_decoder, normalisation, parameter_count)
from oracle.burgers import BurgersFOM, Grid
from oracle.ddmaps import build_dd, restrict, subdomain_residual
from oracle.hyperreduction import greedy_sample, pod_basis, subnet, subnet_decode


# --- Sections 7.5 / 7.6 and their tables: exact integers -------------------------------------------

@pytest.mark.parametrize("nx,ny,sx,sy,expect,total,nA", [
    (480, 24, 2, 2, {(5258, 1006)}, 25056, 2016),
    (480, 24, 2, 1, {(11472, 96)}, 23136, 96),
    (480, 24, 4, 2, {(2618, 526), (2596, 572)}, 25248, 2208),
    (480, 24, 8, 2, {(1298, 286), (1276, 332)}, 25632, 2592),
    (36, 36, 2, 2, {(578, 142)}, 2880, 288),
    (240, 240, 4, 4, {(6962, 478), (6844, 716), (6728, 952)}, 120960, 5760),
])
def test_dd_sizes(nx, ny, sx, sy, expect, total, nA):
    """N_i^Omega = 5258 (printed 5238; forced by 25056 = 4 (5258 + 1006)), N_i^Gamma = 1006,
    25056 aggregated DoF for the 480x24 2x2 split (Section 7.6); the other splits
    reproduce the parameter counts of the subdomain-configuration table."""
    dd = build_dd(Grid(nx, ny), sx, sy)
    assert {(len(s.omega), len(s.gamma)) for s in dd.subdomains} == expect
    assert sum(len(s.omega) + len(s.gamma) for s in dd.subdomains) == total
    assert dd.n_A == nA == total - 2 * nx * ny


def test_dd_structure():
    g = Grid(12, 8)
    dd = build_dd(g, 2, 2)
    rows = np.concatenate([s.res_rows for s in dd.subdomains])
    assert np.array_equal(np.sort(rows), np.arange(g.n_dof))          # non-overlapping, sum N_i^r = N_x
    om = np.concatenate([s.omega for s in dd.subdomains])
    assert len(np.unique(om)) == len(om)                              # P_i^Omega non-overlapping
    # A x_restricted = 0 for every global state; (A_1..A_n) has full row rank
    x = np.random.default_rng(0).standard_normal(g.n_dof)
    c = sum(A @ x[s.gamma] for A, s in zip(dd.A, dd.subdomains))
    assert np.allclose(c, 0)
    Afull = np.hstack([A.toarray() for A in dd.A])
    assert np.linalg.matrix_rank(Afull) == dd.n_A
    assert set(np.unique(Afull)) <= {-1.0, 0.0, 1.0}
    # ports are non-overlapping and sum_j N_j^p = N_i^Gamma for every subdomain
    for s in dd.subdomains:
        n = sum(len(p[1]) for p in dd.ports if s.index in p[0])
        assert n == len(s.gamma)
    # corner ports of a 2x2 five-point split are shared by three subdomains
    assert max(len(p[0]) for p in dd.ports) == 3


def test_dd_residual_identity():
    """r(x) = sum_i (P_i^r)^T r_i(P_i^Omega x, P_i^Gamma x)  (eq. fom_dd_residual)."""
    g = Grid(10, 6)
    f = BurgersFOM(g)
    dd = build_dd(g, 2, 2)
    mu = (40.0, 9.0)
    x = np.random.default_rng(2).standard_normal(g.n_dof)
    r = np.zeros(g.n_dof)
    for i, (xo, xg) in enumerate(restrict(dd, x)):
        r[dd.subdomains[i].res_rows] += subdomain_residual(f, dd, i, xo, xg, mu)
    assert np.allclose(r, f.residual(x, mu), rtol=1e-14, atol=1e-9)


# --- Sections 5.1 / 7.3: mask and parameter counts -----------------------------------

def test_mask_nnz_and_widths():
    """Widths 26290 / 5030 and mask nonzeros 78820 / 15040 for (b, s) = (5, 5) (Section 7.6)."""
    assert band_mask(5258, 5, 5).shape == (5258, 26290)
    assert band_mask(5258, 5, 5).nnz == 78820
    assert band_mask(1006, 5, 5).shape == (1006, 5030)
    assert band_mask(1006, 5, 5).nnz == 15040


def test_parameter_counts():
    """Table of subdomain configurations (Section 7.5), (n^Omega, n^Gamma) = (6, 3),
    (b, s) = (5, 5), 1x1 with n = 9: the largest interior autoencoder per split and the
    total over all interior and interface autoencoders."""
    P = lambda N, n: parameter_count(N, n, 5, 5)
    assert P(23040, 9) == 2995100
    assert P(11472, 6) == 1147100
    assert 2 * (P(11472, 6) + P(96, 3)) == 2307440
    assert P(5258, 6) == 525700
    assert 4 * (P(5258, 6) + P(1006, 3)) == 2384080
    assert max(P(2618, 6), P(2596, 6)) == 261700
    assert 4 * (P(2618, 6) + P(526, 3)) + 4 * (P(2596, 6) + P(572, 3)) == 2391440
    assert max(P(1298, 6), P(1276, 6)) == 129700
    assert 4 * (P(1298, 6) + P(286, 3)) + 12 * (P(1276, 6) + P(332, 3)) == 2406160


def test_encoder_parameter_counts():
    """Dense vs sparse encoder (240x12 grid, n = 4): 99,619,200 and 230,350 parameters."""
    N, n = 5760, 4
    sparse_enc = band_mask(N, 5, 5).nnz + 5 * N + n * 5 * N
    dense_w = 17280
    dense_enc = N * dense_w + dense_w + n * dense_w
    assert sparse_enc == 230350
    assert dense_enc == 99619200


# --- decoder, Jacobian, gradients -----------------------------------------------------

def _random_decoder(N=30, n=4, b=3, s=2, activation=ACT_SIGMOID, seed=0):
    ae = MaskedAE(N, n, b, s, activation)
    p = ae.init_params(seed)
    rng = np.random.default_rng(seed)
    p.W1d = rng.standard_normal(p.W1d.shape)
    p.b1d = 0.3 * rng.standard_normal(p.b1d.shape)
    nm = normalisation(rng.standard_normal((5, N)))
    return ae, p, nm, export_decoder(ae, p, nm)


@pytest.mark.parametrize("activation", [ACT_SIGMOID, ACT_SWISH, ACT_IDENTITY])
def test_decoder_jacobian_fd(activation):
    _, _, _, dec = _random_decoder(activation=activation)
    xh = np.random.default_rng(5).standard_normal(dec.n)
    g0, J = decode_jacobian(dec, xh)
    Jfd = np.zeros_like(J)
    for k in range(dec.n):
        e = np.zeros(dec.n)
        e[k] = 1e-6
        Jfd[:, k] = (decode_jacobian(dec, xh + e)[0] - decode_jacobian(dec, xh - e)[0]) / 2e-6
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * max(1.0, np.max(np.abs(J)))


def test_subnet_equals_full_decoder():
    """The subnet reproduces the selected outputs of the full decoder (Section 5.4)."""
    _, _, _, dec = _random_decoder(N=40, n=5, b=4, s=3)
    I_o = np.array([0, 3, 4, 17, 39])
    sn = subnet(dec, I_o)
    xh = np.random.default_rng(1).standard_normal(5)
    g, J = decode_jacobian(dec, xh)
    gs, Js = subnet_decode(sn, xh)
    assert np.allclose(gs, g[I_o], rtol=1e-14, atol=1e-14)
    assert np.allclose(Js, J[I_o], rtol=1e-14, atol=1e-14)
    assert len(sn.I_h) < dec.w


def test_autoencoder_gradient_fd():
    ae = MaskedAE(12, 3, 2, 2, ACT_SIGMOID)
    p = ae.init_params(3)
    rng = np.random.default_rng(4)
    p.b1d += 0.2 * rng.standard_normal(p.b1d.shape)
    p.b1e += 0.2 * rng.standard_normal(p.b1e.shape)
    X = rng.standard_normal((5, 12))
    scale = rng.uniform(0.5, 2.0, 12)
    loss, grads = ae.forward_backward(p, X, scale)
    assert np.isclose(loss, ae.loss(p, X, scale), rtol=1e-13)
    for name in ("W1e", "b1e", "W2e", "W1d", "b1d", "W2d"):
        arr = getattr(p, name)
        gr = getattr(grads, name)
        flat, gflat = arr.reshape(-1), gr.reshape(-1)
        for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + 1e-6
            lp = ae.loss(p, X, scale)
            flat[k] = old - 1e-6
            lm = ae.loss(p, X, scale)
            flat[k] = old
            assert abs((lp - lm) / 2e-6 - gflat[k]) <= 1e-6 * max(1.0, abs(gflat[k])), name


def test_adam_first_step_closed_form():
    """First Adam step moves each parameter by lr * g / (|g| + eps) (bias-corrected)."""
    x = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -1e-3, 4.0])
    opt = Adam([x], lr=1e-2)
    x0 = x.copy()
    opt.step([x], [g])
    assert np.allclose(x, x0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_normalisation_range():
    X = np.random.default_rng(0).standard_normal((7, 9)) * 3 + 1
    X[:, 2] = 5.0
    nm = normalisation(X)
    Xn = (X - nm.m) / nm.s
    assert np.allclose(Xn[:, [0, 1, 3]].max(0), 1) and np.allclose(Xn[:, [0, 1, 3]].min(0), -1)
    assert np.allclose(Xn[:, 2], 0)


# --- HR -----------------------------------------------------------------------------------

def test_pod_energy_criterion():
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((50, 6)))
    V, _ = np.linalg.qr(rng.standard_normal((8, 6)))
    S = np.array([10.0, 5.0, 1.0, 1e-3, 1e-6, 1e-9])
    X = U @ np.diag(S) @ V.T
    tot = (S ** 2).sum()
    for tol in (1e-1, 1e-4, 1e-10):
        n = pod_basis(X, tol).shape[1]
        assert (S[:n] ** 2).sum() >= (1 - tol) * tot
        assert n == 1 or (S[:n - 1] ** 2).sum() < (1 - tol) * tot


def test_greedy_invariants():
    rng = np.random.default_rng(1)
    n_own = 40
    Phi, _ = np.linalg.qr(rng.standard_normal((2 * n_own, 5)))
    sel = greedy_sample(Phi, n_own, 12)
    assert len(sel) == 12 and len(np.unique(sel)) == 12 and sel.min() >= 0 and sel.max() < n_own
    assert np.array_equal(sel, greedy_sample(Phi, n_own, 12))
    rows = np.concatenate([sel, sel + n_own])
    assert np.linalg.matrix_rank(Phi[rows]) == 5
    # a basis vector supported on one node makes that node the first choice
    P2 = np.zeros((2 * n_own, 1)); P2[7, 0] = 1.0
    assert 7 in greedy_sample(P2, n_own, 1)
