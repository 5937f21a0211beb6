"""Parity of the HIP library (through its C ABI) with the FP64 oracle on identical
seeded inputs.  FP64 mode: relative 1e-12 per kernel, 1e-10 for SQP steps and solves
(latents and multipliers alike, equal iteration counts).
FP32-decoder mode: tolerances derived from FP32 rounding (stated per test)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.autoencoder import decode_jacobian
from oracle.burgers import solve_fom
from oracle.ddmaps import subdomain_residual_jac
from oracle.pack import load_pack
from oracle.rom import (CONVERGED, SQPOptions, evaluate, hr_interior_rows, kkt_matrix, kkt_rhs, relative_error,
                        sqp_solve, sqp_step)


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module", params=["tiny", "cfg0", "tinymix", "tinywide", "tinyl10", "tinyl16"])
def case(request, dr):
    pack = request.getfixturevalue(request.param + "_pack")
    print(f"[case {request.param}]", flush=True)
    return request.param, pack, dr.Model(pack), load_pack(pack)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def test_sizes_and_subnet_rows(case):
    name, pack, gm, om = case
    assert gm.n_D == om.n_D and gm.n_C == om.n_C and gm.N_A == om.dd.n_A
    for i, sd in enumerate(om.dd.subdomains):
        assert gm.N_om[i] == len(sd.omega) and gm.N_ga[i] == len(sd.gamma)
        assert np.array_equal(gm.subnet_rows(i, 0), hr_interior_rows(om, i))     # bit-exact index parity


@pytest.mark.parametrize("B", [1, 70])
def test_decoder_parity(dr, case, B):
    name, pack, gm, om = case
    ws = dr.Workspace(gm, B)
    for i in range(gm.n_sub):
        for part, dec in ((0, om.dec_om[i]), (1, om.dec_ga[i])):
            rows = gm.subnet_rows(i, part)
            xh = si.normal((B, dec.n), seed=100 + 7 * i + part, scale=1.5)
            x, J = dr.ae_jacobian_hr(gm, ws, i, part, xh, precision=dr.PREC_FP64)
            x, J = x.cpu().numpy(), J.cpu().numpy()
            x32, J32 = dr.ae_jacobian_hr(gm, ws, i, part, xh, precision=dr.PREC_FP32_DECODER)
            x32, J32 = x32.cpu().numpy(), J32.cpu().numpy()
            xd = dr.ae_decode_hr(gm, ws, i, part, xh, precision=dr.PREC_FP64).cpu().numpy()
            for b in range(B):
                g, Jr = decode_jacobian(dec, xh[b])
                assert relerr(x[b], g[rows]) <= 1e-13
                assert relerr(xd[b], g[rows]) <= 1e-13
                assert relerr(J[b], Jr[rows]) <= 1e-12
                # FP32: 27-term band sums of O(1) terms, relative to the row scale
                assert relerr(x32[b], g[rows]) <= 2e-6
                assert relerr(J32[b], Jr[rows]) <= 2e-5


def test_dd_fom_residual_parity(dr, case):
    name, pack, gm, om = case
    B = 3
    mus = si.heldout_mu(B, 5)
    rng = np.random.default_rng(0)
    xs = []
    for b in range(B):
        x = om.fom.exact_state(mus[b]) + 0.01 * rng.standard_normal(om.grid.n_dof)
        xs.append(np.concatenate([np.concatenate([x[sd.omega], x[sd.gamma]]) for sd in om.dd.subdomains]))
    r, Jv = dr.dd_fom_residual(gm, mus, np.stack(xs), jac=True)
    r, Jv = r.cpu().numpy(), Jv.cpu().numpy()
    g = om.grid
    for b in range(B):
        off = 0
        ref, refJ = [], []
        for i, sd in enumerate(om.dd.subdomains):
            xo = xs[b][off:off + len(sd.omega)]
            xg = xs[b][off + len(sd.omega):off + len(sd.omega) + len(sd.gamma)]
            off += len(sd.omega) + len(sd.gamma)
            ri, dro, drg = subdomain_residual_jac(om.fom, om.dd, i, xo, xg, mu=mus[b])
            ref.append(ri)
            # Jacobian entries in the fixed slot order, from the oracle's sparse Jacobian
            n_own = len(sd.own_nodes)
            for f in (0, 1):
                for p, q in enumerate(sd.own_nodes):
                    j, ii = divmod(int(q), g.nx)
                    row = np.zeros(6)
                    nbrs = [(ii, j), (ii - 1, j), (ii + 1, j), (ii, j - 1), (ii, j + 1)]
                    for t, (a, c) in enumerate(nbrs):
                        if 0 <= a < g.nx and 0 <= c < g.ny:
                            col = c * g.nx + a + f * g.n_nodes
                            row[t] = _dd_entry(dro, drg, sd, p + f * n_own, col)
                    other = q + (1 - f) * g.n_nodes
                    row[5] = _dd_entry(dro, drg, sd, p + f * n_own, other)
                    refJ.append(row)
        ref = np.concatenate(ref)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(r[b] - ref)) <= 1e-12 * max(scale, 1.0) * 1e2
        assert relerr(Jv[b], np.array(refJ)) <= 1e-13


def _dd_entry(dro, drg, sd, row, col):
    k = np.searchsorted(sd.omega, col)
    if k < len(sd.omega) and sd.omega[k] == col:
        return dro[row, k]
    k = np.searchsorted(sd.gamma, col)
    return drg[row, k]


def test_gn_blocks_parity(dr, case):
    name, pack, gm, om = case
    B = 5
    mus = si.heldout_mu(B, 9)
    xh = si.normal((B, gm.n_D), seed=3, scale=0.5)
    ws = dr.Workspace(gm, B)
    H, g, EG, c, rr = (t.cpu().numpy() for t in dr.gn_blocks(gm, ws, mus, xh, precision=dr.PREC_FP64))
    for b in range(B):
        ev = evaluate(om, mus[b], xh[b])
        for i, (o, (a, m)) in enumerate(zip(om.offsets(), om.sizes())):
            assert relerr(H[b, i, :a + m, :a + m], ev.H[i]) <= 1e-11
            assert relerr(g[b, o:o + a + m], ev.g[i]) <= 1e-10
            assert relerr(EG[b, i, :, :m], ev.EG[i]) <= 1e-12
        assert relerr(c[b], ev.c) <= 1e-12
        assert relerr(rr[b], sum(float(z @ z) for z in ev.Zr)) <= 1e-11


def test_sqp_step_parity(dr, case):
    name, pack, gm, om = case
    B = 4
    mus = si.heldout_mu(B, 13)
    xh = si.normal((B, gm.n_D), seed=4, scale=0.2)
    lam = si.normal((B, gm.n_C), seed=5, scale=0.01)
    ws = dr.Workspace(gm, B)
    o = dr.opts(precision=dr.PREC_FP64, max_backtracks=20)
    x1, l1, fn, st = (t.cpu().numpy() for t in dr.sqp_step(gm, ws, mus, xh, lam, o))
    for b in range(B):
        xr, lr, _, fr, sr, _, _ = sqp_step(om, mus[b], xh[b], lam[b], SQPOptions(max_backtracks=20))
        kap = np.linalg.cond(kkt_matrix(om, evaluate(om, mus[b], xh[b])))
        print(name, b, "step x err %.2e lam err %.2e cond(K) %.2e" % (relerr(x1[b], xr), relerr(l1[b], lr), kap),
              flush=True)
        assert int(st[b]) == (1 if sr == -1 else sr)
        assert relerr(x1[b], xr) <= 1e-10
        assert relerr(l1[b], lr) <= 1e-10
        assert abs(fn[b] - fr) <= 1e-10 * max(1.0, fr)


@pytest.mark.parametrize("B", [1, 5])
def test_rom_solve_parity(dr, case, B):
    name, pack, gm, om = case
    mus = si.heldout_mu(B, 17)
    ws = dr.Workspace(gm, B)
    o = dr.opts(max_iter=100, tol_rel=1e-12, precision=dr.PREC_FP64)
    out = dr.rom_solve_batch(gm, ws, mus, o)
    out = {k: v.cpu().numpy() for k, v in out.items()}
    for b in range(B):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-12))
        ev = evaluate(om, mus[b], ref.xhat)
        kap = np.linalg.cond(kkt_matrix(om, ev))
        print(name, b, "status", out["status"][b], ref.status, "iters", out["iters"][b], ref.iters,
              "x err %.2e lam err %.2e cond(K) %.2e |F|/|F0| %.2e" % (
                  relerr(out["xhat"][b], ref.xhat), relerr(out["lam"][b][:gm.n_C], ref.lam), kap,
                  ref.fnorm / ref.fnorm0), flush=True)
        assert int(out["status"][b]) == ref.status
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        assert relerr(out["lam"][b][:gm.n_C], ref.lam) <= 1e-10
        assert int(out["iters"][b]) == ref.iters
        assert abs(out["fnorm0"][b] - ref.fnorm0) <= 1e-12 * ref.fnorm0


def test_rom_solve_repeat_and_reuse(dr, case):
    """A cached graph replayed for a second batch gives the same results as a fresh one."""
    name, pack, gm, om = case
    mus = si.heldout_mu(6, 23)
    ws = dr.Workspace(gm, 6)
    o = dr.opts(max_iter=60, tol_rel=1e-9, precision=dr.PREC_FP64)
    a = dr.rom_solve_batch(gm, ws, mus, o)["xhat"].cpu().numpy()
    b = dr.rom_solve_batch(gm, ws, mus[::-1].copy(), o)["xhat"].cpu().numpy()
    c = dr.rom_solve_batch(gm, ws, mus, o)["xhat"].cpu().numpy()
    assert np.array_equal(a, c)
    assert np.array_equal(a, b[::-1])


def test_fp32_decoder_solve(dr, case):
    """FP32 decoders, FP64 residual/KKT: the solve stops at the FP32 noise floor; its
    error against the FOM stays within 10% (plus 1e-4 absolute) of the FP64 solve's."""
    name, pack, gm, om = case
    B = 3
    mus = si.heldout_mu(B, 29)
    ws = dr.Workspace(gm, B)
    o64 = dr.opts(max_iter=60, tol_rel=1e-8, precision=dr.PREC_FP64)
    o32 = dr.opts(max_iter=60, tol_rel=1e-6, precision=dr.PREC_FP32_DECODER)
    x64 = dr.rom_solve_batch(gm, ws, mus, o64)["xhat"].cpu().numpy()
    r32 = dr.rom_solve_batch(gm, ws, mus, o32)
    x32 = r32["xhat"].cpu().numpy()
    for b in range(B):
        xf = solve_fom(om.fom, mus[b]).x
        e64 = relative_error(om, x64[b], xf)
        e32 = relative_error(om, x32[b], xf)
        print(name, b, "rel err fp64 %.3e fp32 %.3e status %d" % (e64, e32, int(r32["status"][b])), flush=True)
        assert e32 <= 1.1 * e64 + 1e-4
