"""Pins of the strong ROM-port constraint (SRPC) oracle (Section 3.2 and Section 5.2):
the interface decoder implied by the port decoders (eq. gamma_map_port) equals the block-form
decoder assembled from the same weights (eq. interface_decoder_rom_port_blocks), its Jacobian
matches central differences, Theorem 3 (i) on the constraint matrix, strong compatibility of
the FOM ports on the feasible set, the port latent-size rule, and the SQP's linear constraint."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.autoencoder import ACT_SIGMOID, Decoder, act, band_columns
from oracle.burgers import Grid
from oracle.ddmaps import build_dd
from oracle.rom import CONVERGED, SQPOptions, evaluate, kkt_rhs, sqp_solve, sqp_step
from oracle.srpc import build_port_maps, interface_decoders, port_latent_size


def _port_decoders(dd, n_tilde, seed, b=3, s=3):
    rng = np.random.default_rng(seed)
    out = []
    for car, dofs in dd.ports:
        N = len(dofs)
        n = port_latent_size(N, n_tilde)
        w = N * s
        out.append(Decoder(0.7 * rng.standard_normal((w, n)), 0.2 * rng.standard_normal(w),
                           0.3 * rng.standard_normal((N, 3, b)), rng.standard_normal(N), b, s, ACT_SIGMOID))
    return out


@pytest.mark.parametrize("split", [(2, 2), (3, 2), (2, 1)])
def test_port_latent_rule_and_theorem3(split):
    """n_j^p = max(min(N_j^p - 1, n~), 1) (Section 7.6): a one-node port (two DoFs) gets one
    latent; Theorem 3 (i): (Ahat_1, ..., Ahat_n) has full row rank n_A = sum_j (|P(j)| - 1) n_j^p
    and a null space of dimension sum_i n_i^Gamma - n_A >= 1."""
    dd = build_dd(Grid(12, 8), *split)
    for n_tilde in (1, 2, 5):
        n_p = [port_latent_size(len(d), n_tilde) for _, d in dd.ports]
        for (car, d), n in zip(dd.ports, n_p):
            assert 1 <= n < len(d) or len(d) == 1
            if len(d) == 2:
                assert n == 1
        pm = build_port_maps(dd, n_p)
        assert pm.n_A == sum((len(c) - 1) * n for (c, _), n in zip(dd.ports, n_p))
        A = np.hstack(pm.A_hat)
        assert set(np.unique(A)) <= {-1.0, 0.0, 1.0}
        assert np.linalg.matrix_rank(A) == pm.n_A
        assert A.shape[1] - pm.n_A >= 1 and A.shape[1] == sum(pm.n_ga)
        # reduced interface size: the copies of every port the subdomain carries
        for i in range(dd.n_sub):
            assert pm.n_ga[i] == sum(n_p[j] for j, (c, _) in enumerate(dd.ports) if i in c)


def test_interface_decoder_equals_block_form():
    """eq. gamma_map_port (sum over ports of P^T g_j^p(Phat xhat)) against the decoder
    x_ref + W2 sigma(W1 xhat + b1) with W1, b1, W2 and the activation assembled in the block
    form of eq. interface_decoder_rom_port_blocks (plus the ports' output offsets, stacked the
    same way); values and Jacobians, the latter also against central differences."""
    dd = build_dd(Grid(12, 8), 2, 2)
    pdec = _port_decoders(dd, 2, seed=3)
    pm = build_port_maps(dd, [d.n for d in pdec])
    gdec = interface_decoders(dd, pm, pdec)
    rng = np.random.default_rng(4)
    for i, sd in enumerate(dd.subdomains):
        Q = pm.Q[i]
        Ng, ng = len(sd.gamma), pm.n_ga[i]
        # block form: W1 = blockdiag(W1^{g_j}) [Phat_i^{j_1}; ...], W2 = [P^{j_1 T} ...] blockdiag(W2^{g_j})
        ws = [pdec[j].w for j in Q]
        W1 = np.zeros((sum(ws), ng))
        b1 = np.concatenate([pdec[j].b1 for j in Q])
        W2 = np.zeros((Ng, sum(ws)))
        xref = np.zeros(Ng)
        h0 = 0
        for j, w in zip(Q, ws):
            Phat = np.zeros((pdec[j].n, ng))
            Phat[np.arange(pdec[j].n), pm.lat_off[i][j] + np.arange(pdec[j].n)] = 1.0
            W1[h0:h0 + w] = pdec[j].W1 @ Phat
            P = np.zeros((pdec[j].N, Ng))
            P[np.arange(pdec[j].N), pm.rows[i][j]] = 1.0
            W2[:, h0:h0 + w] = P.T @ pdec[j].W2().toarray()
            xref += P.T @ pdec[j].x_ref
            h0 += w
        for _ in range(3):
            x = rng.standard_normal(ng)
            a, da = act(W1 @ x + b1, ACT_SIGMOID)
            g_ref = xref + W2 @ a
            J_ref = W2 @ (da[:, None] * W1)
            g, J = gdec[i].decode_jacobian(x)
            assert np.allclose(g, g_ref, rtol=1e-13, atol=1e-13)
            assert np.allclose(J, J_ref, rtol=1e-13, atol=1e-13)
            assert np.array_equal(gdec[i].decode(x), g)
            h = 1e-6
            Jfd = np.stack([(gdec[i].decode(x + h * e) - gdec[i].decode(x - h * e)) / (2 * h) for e in np.eye(ng)], 1)
            assert np.max(np.abs(Jfd - J)) <= 1e-7 * max(1.0, np.max(np.abs(J)))


def test_strong_compatibility_on_feasible_set():
    """Where sum_i Ahat_i xhat_i^Gamma = 0, the decoded interface states satisfy the FOM port
    conditions sum_i A_i g_i^Gamma(xhat_i^Gamma) = 0 (Section 3.2) - exactly, since every copy of
    a port latent then feeds the same port decoder the same input."""
    dd = build_dd(Grid(18, 12), 3, 2)
    pdec = _port_decoders(dd, 2, seed=5)
    pm = build_port_maps(dd, [d.n for d in pdec])
    gdec = interface_decoders(dd, pm, pdec)
    rng = np.random.default_rng(6)
    # a feasible point: one value per port, copied into every carrier
    port_val = [rng.standard_normal(d.n) for d in pdec]
    xg = []
    for i in range(dd.n_sub):
        v = np.zeros(pm.n_ga[i])
        for j in pm.Q[i]:
            v[pm.lat_off[i][j]:pm.lat_off[i][j] + pdec[j].n] = port_val[j]
        xg.append(v)
    assert np.max(np.abs(sum(A @ v for A, v in zip(pm.A_hat, xg)))) == 0.0
    resid = sum(dd.A[i] @ gdec[i].decode(xg[i]) for i in range(dd.n_sub))
    assert np.max(np.abs(resid)) == 0.0
    # and an infeasible point violates them
    xg[0] = xg[0] + 0.1
    resid = sum(dd.A[i] @ gdec[i].decode(xg[i]) for i in range(dd.n_sub))
    assert np.max(np.abs(resid)) > 1e-3


def _srpc_model():
    from oracle.build_model import build
    from oracle.pack import load_pack
    pack, *_ = build("tinysrpc2x1", workers=1, verbose=False)
    return load_pack(pack)


def test_srpc_linear_constraint_and_kkt():
    """The constraint Jacobian is the constant Ahat, c is linear in the latents (checked
    against central differences of evaluate()); after an accepted full step from any point the
    constraint holds to rounding (the linearisation of a linear constraint is exact); at
    convergence stationarity and feasibility hold."""
    m = _srpc_model()
    mu = si.heldout_mu(1, 11)[0]
    rng = np.random.default_rng(8)
    x = 0.2 * rng.standard_normal(m.n_D)
    ev = evaluate(m, mu, x)
    h = 1e-6
    for k in rng.choice(m.n_D, 6, replace=False):
        e = np.zeros(m.n_D)
        e[k] = h
        dc = (evaluate(m, mu, x + e).c - evaluate(m, mu, x - e).c) / (2 * h)
        ref = np.zeros(m.n_C)
        for i, (o, (a, b)) in enumerate(zip(m.offsets(), m.sizes())):
            if o + a <= k < o + a + b:
                ref = m.A_hat[i][:, k - o - a]
        assert np.max(np.abs(dc - ref)) <= 1e-8
    lam = rng.standard_normal(m.n_C)
    x1, l1, ev1, f1, st, nb, alpha = sqp_step(m, mu, x, lam, SQPOptions())
    if st == -1 and alpha == 1.0:
        assert np.max(np.abs(ev1.c)) <= 1e-12 * max(1.0, np.max(np.abs(x)))
    res = sqp_solve(m, mu, opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-10))
    assert res.status == CONVERGED, res.status
    F = kkt_rhs(m, evaluate(m, mu, res.xhat), res.lam)
    assert np.linalg.norm(F[:m.n_D]) <= 1e-9 * res.fnorm0
    assert np.max(np.abs(F[m.n_D:])) <= 1e-12 * max(1.0, np.max(np.abs(res.xhat)))
