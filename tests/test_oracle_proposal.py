"""Pins of the proposal oracle: gradient by central differences, closed forms of the input
map, SiLU derivative and the first Adam step, a fit of a known map, and the fallback rule
(it never starts from a point with a larger first KKT residual than the zero start)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import proposal as P
from oracle.autoencoder import Adam
from oracle.rom import SQPOptions, CONVERGED, sqp_solve, sqp_solve_warm


def _net(sizes, seed):
    net = P.mlp_from_init(si.mlp_init(sizes, seed))
    # non-zero biases so that their gradient is exercised
    g = si.rng(seed + 1)
    for k, (W, b) in enumerate(net.layers):
        b[:] = g.uniform(-0.3, 0.3, size=b.shape)
    return net


def test_encode_inputs_maps_box_corners():
    mu = np.array([[1.0, 5.0], [1e4, 20.0], [100.0, 12.5]])
    X = P.encode_inputs(mu)
    assert np.allclose(X, [[-1.0, -1.0], [1.0, 1.0], [0.0, 0.0]], atol=1e-15)


def test_silu_prime_central_difference():
    z = np.linspace(-8, 8, 41)
    h = 1e-6
    fd = (P.silu(z + h) - P.silu(z - h)) / (2 * h)
    assert np.allclose(P.silu_prime(z), fd, rtol=1e-8, atol=1e-10)
    # SiLU(0) = 0, SiLU'(0) = 1/2
    assert P.silu(np.array(0.0)) == 0.0 and P.silu_prime(np.array(0.0)) == 0.5


def test_mlp_gradient_central_differences():
    net = _net([2, 7, 5, 4], 11)
    g = si.rng(3)
    X = g.uniform(-1, 1, size=(6, 2))
    T = g.normal(size=(6, 4))
    loss, grads = net.loss_and_grad(X, T)
    params = net.params()
    for pi, (p, gr) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 6)):
            old = flat[idx]
            h = 1e-6 * max(1.0, abs(old))
            flat[idx] = old + h
            lp = net.loss_and_grad(X, T)[0]
            flat[idx] = old - h
            lm = net.loss_and_grad(X, T)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(gr.reshape(-1)[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (pi, idx)


def test_adam_first_step_closed_form():
    # after one step m/c1 = g and v/c2 = g^2, so the update is -lr g / (|g| + eps)
    w = np.array([0.5, -1.0, 2.0])
    g = np.array([1e-3, -4.0, 0.0])
    opt = Adam([w], lr=1e-3)
    w0 = w.copy()
    opt.step([w], [g])
    assert np.allclose(w - w0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_standardiser_round_trip_and_constant_column():
    g = si.rng(5)
    Y = g.normal(size=(50, 4)) * np.array([1.0, 10.0, 1e-3, 0.0]) + np.array([0.0, 3.0, -2.0, 7.0])
    st = P.standardiser(Y)
    Yn = st.forward(Y)
    assert np.allclose(Yn[:, :3].mean(axis=0), 0.0, atol=1e-10)   # column 2: offset/scale = 2e3
    assert np.allclose(Yn[:, :3].std(axis=0), 1.0, atol=1e-12)
    assert st.std[3] == 1.0 and np.allclose(Yn[:, 3], 0.0)
    assert np.allclose(st.inverse(Yn), Y, atol=1e-12)


def test_training_fits_a_smooth_map():
    # a smooth target on the input box is fitted far below its variance
    g = si.rng(9)
    U = g.uniform(-1, 1, size=(256, 2))
    T = np.stack([np.sin(1.5 * U[:, 0]) + 0.5 * U[:, 1], U[:, 0] * U[:, 1], np.cos(U[:, 1])], axis=1)
    st = P.standardiser(T)
    Tn = st.forward(T)
    net = P.mlp_from_init(si.mlp_init([2, 32, 32, 3], 4))
    tr, te = si.train_split(256, 0.1, 2)
    rep = P.train_proposal(net, U, Tn, tr, te, epochs=150, batch=32, seed=6, lr=3e-3, order_fn=si.epoch_order)
    assert rep.history[-1] < 0.02 * rep.history[0]
    assert rep.test_loss < 0.05


def test_fallback_rule_logic():
    assert not P.use_zero_start(1.0, 2.0)
    assert not P.use_zero_start(2.0, 2.0)
    assert P.use_zero_start(3.0, 2.0)
    assert P.use_zero_start(np.nan, 2.0)
    assert P.use_zero_start(np.inf, 2.0)


def test_warm_start_fallback_and_exact_proposal(tiny_pack):
    from oracle.pack import load_pack
    model = load_pack(tiny_pack)
    mu = si.heldout_mu(1, 0)[0]
    opts = SQPOptions(max_iter=50, tol_abs=0.0, tol_rel=1e-10)
    cold = sqp_solve(model, mu, opts=opts)
    assert cold.status == CONVERGED
    # zero latents with a non-least-squares multiplier: same constraint value as the zero start,
    # larger interface rows of rho (lambda_LS minimises them), so it is rejected
    bad_x = np.zeros(model.n_D)
    bad_l = np.full(model.n_C, 1e3)
    res, fb, f_zero, f_prop = sqp_solve_warm(model, mu, bad_x, bad_l, opts)
    assert fb and f_prop > f_zero
    assert res.iters == cold.iters and np.array_equal(res.xhat, cold.xhat)
    # the converged solution as proposal: accepted, already below tolerance
    res2, fb2, f_zero2, f_prop2 = sqp_solve_warm(model, mu, cold.xhat, cold.lam, opts)
    assert not fb2 and f_prop2 <= f_zero2
    assert res2.status == CONVERGED and res2.iters == 0
    assert f_zero2 == pytest.approx(cold.fnorm0, rel=1e-14)
