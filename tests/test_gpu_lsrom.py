"""LS-ROM (Section 3.3) on the GPU, through the C ABI: the POD maps x = Phi xhat run as dense
decoders with the identity activation (W1 = I, b1 = 0, W2 = Phi) on the same kernels, against
the independent LS-ROM oracle (its own residual route, null-space QP steps) with collocation or
gappy-POD HR (Section 3.1, B_i = (Z_i Phi_i^r)^+ Z_i) on the same nodes: maps and their constant
Jacobians, Gauss-Newton blocks of the hyper-reduced objective, FP64 solves (statuses, iteration
counts, latents and multipliers to 1e-10) and FP32-map solves against the FOM."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle import lsrom
from oracle.burgers import solve_fom
from oracle.pack import load_ls_pack


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module", params=["tinyls", "cfg0ls", "tinylsg", "cfg0lsg"])
def case(request, dr):
    pack = request.getfixturevalue(request.param + "_pack")
    print(f"[lsrom case {request.param}]", flush=True)
    return request.param, pack, dr.Model(pack), load_ls_pack(pack)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def test_lsrom_maps(dr, case):
    """Kept rows of x0 + Phi xhat and their Jacobian rows Phi (interior subnet rows, every
    interface row)."""
    name, pack, gm, rom = case
    B = 70
    ws = dr.Workspace(gm, B)
    for i in range(gm.n_sub):
        for part, (x0, Phi) in ((0, (rom.x0_om[i], rom.Phi_om[i])), (1, (rom.x0_ga[i], rom.Phi_ga[i]))):
            rows = gm.subnet_rows(i, part)
            xh = si.normal((B, Phi.shape[1]), seed=900 + 3 * i + part)
            x, J = (t.cpu().numpy() for t in dr.ae_jacobian_hr(gm, ws, i, part, xh, precision=dr.PREC_FP64))
            for b in range(B):
                assert relerr(x[b], (x0 + Phi @ xh[b])[rows]) <= 1e-13
                assert relerr(J[b], Phi[rows]) <= 1e-15


def test_lsrom_gn_blocks(dr, case):
    """H_i = J_i^T J_i, g_i = J_i^T (B_i r_i) and the summed squares of the hyper-reduced residual
    B_i r_i (collocation: the sampled rows; gappy POD: their projection) against the oracle's
    stacked residual and Jacobian."""
    name, pack, gm, rom = case
    B = 5
    mus = si.heldout_mu(B, 9)
    xh = si.normal((B, gm.n_D), seed=3, scale=0.5)
    ws = dr.Workspace(gm, B)
    H, g, EG, c, rr = (t.cpu().numpy() for t in dr.gn_blocks(gm, ws, mus, xh, precision=dr.PREC_FP64))
    for b in range(B):
        r, J = rom.residual(mus[b], xh[b])
        o_r, o_x, rr_ref = 0, 0, 0.0
        for i, (a, m) in enumerate(rom.sizes):
            k = rom.hr[i].P.shape[0] if rom.hr[i].P is not None else len(rom.hr[i].rows)
            ri, Ji = r[o_r:o_r + k], J[o_r:o_r + k, o_x:o_x + a + m]
            assert relerr(H[b, i, :a + m, :a + m], Ji.T @ Ji) <= 1e-11
            assert relerr(g[b, o_x:o_x + a + m], Ji.T @ ri) <= 1e-10
            rr_ref += float(ri @ ri)
            o_r += k
            o_x += a + m
        assert o_r == len(r)
        assert relerr(rr[b], rr_ref) <= 1e-11


@pytest.mark.parametrize("B", [1, 6])
def test_lsrom_solve(dr, case, B):
    name, pack, gm, rom = case
    mus = si.heldout_mu(B, 17)
    ws = dr.Workspace(gm, B)
    out = {k: v.cpu().numpy() for k, v in dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=100, tol_rel=1e-12,
                                                                                  precision=dr.PREC_FP64)).items()}
    for b in range(B):
        ref = lsrom.solve(rom, mus[b], max_iter=100, tol_abs=0.0, tol_rel=1e-12)
        print(name, b, "status", out["status"][b], ref.status, "iters", out["iters"][b], ref.iters,
              "x err %.2e lam err %.2e" % (relerr(out["xhat"][b], ref.xhat), relerr(out["lam"][b][:gm.n_C], ref.lam)),
              flush=True)
        assert int(out["status"][b]) == ref.status and int(out["iters"][b]) == ref.iters
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        assert relerr(out["lam"][b][:gm.n_C], ref.lam) <= 1e-10
        assert abs(out["fnorm0"][b] - ref.fnorm0) <= 1e-12 * ref.fnorm0


def test_lsrom_fp32_maps(dr, case):
    """FP32 maps, FP64 residual and KKT: error against the FOM within 10% (plus 1e-4) of the
    FP64 solve's."""
    name, pack, gm, rom = case
    B = 3
    mus = si.heldout_mu(B, 29)
    ws = dr.Workspace(gm, B)
    x64 = dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=60, tol_rel=1e-8, precision=dr.PREC_FP64))["xhat"]
    x32 = dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=60, tol_rel=1e-6, precision=dr.PREC_FP32_DECODER,
                                                  stall_tol=1e-5, stall_ratio=0.5))["xhat"]
    f = dict(dtype=torch.float64, device="cuda")
    xf = torch.as_tensor(np.stack([solve_fom(rom.fom, m).x for m in mus]), **f)
    e64 = dr.relative_error(gm, ws, x64, xf).cpu().numpy()
    e32 = dr.relative_error(gm, ws, x32, xf).cpu().numpy()
    for b in range(B):
        print(name, b, "rel err fp64 %.3e fp32 %.3e" % (e64[b], e32[b]), flush=True)
        assert e32[b] <= 1.1 * e64[b] + 1e-4


def test_gappy_blocks_at_benchmark_size(dr):
    """Gappy POD at the benchmark's grid and split (240x240, 4x4, POD maps (8,4), 360 sampled
    nodes: 720 stored rows and 12-15 modes per subdomain, so the projection takes several row
    chunks and mode tiles) over two 64-solve groups: GN blocks of sampled lanes and two FP64
    solves against the oracle.  At this size the zero start's KKT residual is about 1e14 and the
    solves stop near 1e3 (tolerance 1e-10 relative), so the two sides' latents, formed by
    different KKT routes, agree to rounding amplified by that range: 7.8e-10 measured, bound
    1e-8; the blocks themselves agree to 1e-11."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "models", "cfg1lsg.npz")
    if not os.path.exists(path):
        pytest.skip("models/cfg1lsg.npz not built")
    pack = dict(np.load(path, allow_pickle=False))
    gm, rom = dr.Model(pack), load_ls_pack(pack)
    assert max(h.P.shape[0] for h in rom.hr) > 8 and max(h.P.shape[1] for h in rom.hr) > 256
    B = 70
    print("[gappy 240x240 4x4] GN blocks, B = 70", flush=True)
    mus = si.heldout_mu(B, 41)
    xh = si.normal((B, gm.n_D), seed=43, scale=0.5)
    ws = dr.Workspace(gm, B)
    H, g, EG, c, rr = (t.cpu().numpy() for t in dr.gn_blocks(gm, ws, mus, xh, precision=dr.PREC_FP64))
    for b in (0, 37, 69):
        r, J = rom.residual(mus[b], xh[b])
        o_r, o_x, rr_ref = 0, 0, 0.0
        for i, (a, m) in enumerate(rom.sizes):
            k = rom.hr[i].P.shape[0]
            ri, Ji = r[o_r:o_r + k], J[o_r:o_r + k, o_x:o_x + a + m]
            assert relerr(H[b, i, :a + m, :a + m], Ji.T @ Ji) <= 1e-11
            assert relerr(g[b, o_x:o_x + a + m], Ji.T @ ri) <= 1e-10
            rr_ref += float(ri @ ri)
            o_r += k
            o_x += a + m
        assert relerr(rr[b], rr_ref) <= 1e-11
    print("[gappy 240x240 4x4] FP64 solves, B = 2", flush=True)
    mus = si.heldout_mu(2, 47)
    ws = dr.Workspace(gm, 2)
    out = {k: v.cpu().numpy() for k, v in dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=40, tol_rel=1e-10,
                                                                                  precision=dr.PREC_FP64)).items()}
    for b in range(2):
        ref = lsrom.solve(rom, mus[b], max_iter=40, tol_abs=0.0, tol_rel=1e-10)
        print("gappy 240x240", b, "status", out["status"][b], ref.status, "iters", out["iters"][b], ref.iters,
              "x err %.2e" % relerr(out["xhat"][b], ref.xhat), flush=True)
        assert int(out["status"][b]) == ref.status and int(out["iters"][b]) == ref.iters
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-8
