"""Pins of the gappy-POD hyper-reduction operator B_i = (Z_i Phi_i^r)^+ Z_i (Section 3.1) in the
LS-ROM oracle, against what the mathematics fixes:
  * the pseudo-inverse inverts the sampled basis: B_i Phi_i^r = I when Z_i Phi_i^r has full
    column rank, so a residual in the basis' span is recovered exactly (Phi_i^r B_i r = r);
  * every residual row sampled and an orthonormal basis of the whole residual space: B_i is
    orthogonal, ||B_i r_i|| = ||r_i||, and the gappy LS-ROM takes the same iterates as the
    LS-ROM without hyper-reduction;
  * the objective depends on the basis' span only: rotating Phi_i^r inside it leaves the
    iterates unchanged."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import lsrom
from oracle.lsrom import HROperator, collocation_operator, gappy_pod_operator
from oracle.pack import load_ls_pack


@pytest.fixture(scope="module")
def tinylsg():
    from oracle.build_model import build
    pack, *_ = build("tinylsg", workers=1, verbose=False)
    return pack


def test_pseudo_inverse_recovers_span(tinylsg):
    rom = load_ls_pack(tinylsg)
    g = si.rng(3)
    for i, sd in enumerate(rom.dd.subdomains):
        nodes = np.sort(np.asarray(tinylsg[f"hr{i}"], dtype=np.int64))
        Phi = np.linalg.qr(g.normal(size=(len(sd.res_rows), 5)))[0]
        op = gappy_pod_operator(rom.dd.grid, nodes, sd.res_rows, Phi)
        pos = {int(r): k for k, r in enumerate(sd.res_rows)}
        ZPhi = Phi[[pos[int(r)] for r in op.rows]]
        assert np.allclose(op.P @ ZPhi, np.eye(5), atol=1e-12)
        r = Phi @ g.normal(size=5)                       # a residual in the span
        rz = r[[pos[int(q)] for q in op.rows]]
        assert np.allclose(Phi @ (op.P @ rz), r, atol=1e-12)
        # the loaded pack's operators have the shape (n_r, 2 N_B) and the same property
        P = np.asarray(tinylsg[f"gp{i}_P"])
        assert P.shape[1] == 2 * len(nodes) and P.shape[0] <= P.shape[1]


def _solve_all(rom, mus):
    return [lsrom.solve(rom, mu, max_iter=60, tol_abs=0.0, tol_rel=1e-12) for mu in mus]


def test_full_sampling_orthonormal_basis_is_no_hr(tinylsg):
    base = load_ls_pack(tinylsg, use_hr=False)
    g = si.rng(5)
    hr = []
    for sd in base.dd.subdomains:
        Q = np.linalg.qr(g.normal(size=(len(sd.res_rows), len(sd.res_rows))))[0]
        hr.append(gappy_pod_operator(base.dd.grid, sd.own_nodes, sd.res_rows, Q))
    full = lsrom.LSROM(base.fom, base.dd, base.C, base.x0_om, base.Phi_om, base.x0_ga, base.Phi_ga, hr=hr)
    mus = si.heldout_mu(3, 21)
    for a, b in zip(_solve_all(full, mus), _solve_all(base, mus)):
        assert a.status == b.status == lsrom.CONVERGED and a.iters == b.iters
        assert np.max(np.abs(a.xhat - b.xhat)) <= 1e-9 * np.max(np.abs(b.xhat))
        assert np.max(np.abs(a.lam - b.lam)) <= 1e-8 * np.max(np.abs(b.lam))


def test_rotation_inside_the_span(tinylsg):
    rom = load_ls_pack(tinylsg)
    g = si.rng(7)
    hr = []
    for op in rom.hr:
        k = op.P.shape[0]
        Q = np.linalg.qr(g.normal(size=(k, k)))[0]
        hr.append(HROperator(op.rows, Q.T @ op.P))     # basis Phi Q: pseudo-inverse Q^T (Z Phi)^+
    rot = lsrom.LSROM(rom.fom, rom.dd, rom.C, rom.x0_om, rom.Phi_om, rom.x0_ga, rom.Phi_ga, hr=hr)
    mus = si.heldout_mu(3, 23)
    for a, b in zip(_solve_all(rot, mus), _solve_all(rom, mus)):
        assert a.status == b.status and a.iters == b.iters
        assert np.max(np.abs(a.xhat - b.xhat)) <= 1e-9 * np.max(np.abs(b.xhat))


def test_gappy_differs_from_collocation(tinylsg):
    """A gappy operator that is not an isometry on the sampled rows changes the objective (so
    the two HR types are not silently the same path)."""
    rom = load_ls_pack(tinylsg)
    col = lsrom.LSROM(rom.fom, rom.dd, rom.C, rom.x0_om, rom.Phi_om, rom.x0_ga, rom.Phi_ga,
                      hr=[collocation_operator(rom.dd.grid, np.asarray(tinylsg[f"hr{i}"], np.int64))
                          for i in range(len(rom.hr))])
    mu = si.heldout_mu(1, 25)[0]
    a, b = lsrom.solve(rom, mu, max_iter=60, tol_abs=0.0, tol_rel=1e-12), lsrom.solve(col, mu, max_iter=60,
                                                                                       tol_abs=0.0, tol_rel=1e-12)
    assert np.max(np.abs(a.xhat - b.xhat)) > 1e-6 * np.max(np.abs(b.xhat))
