"""Strong ROM-port constraint formulation on the GPU (through the C ABI) against the FP64 oracle:
interface decoders assembled from port decoders (eq. gamma_map_port), the linear constraint
sum_i Ahat_i xhat_i^Gamma with its constant Jacobian, Gauss-Newton blocks, one SQP step, full
solves (FP64 to 1e-10; FP32 decoders within 10% of the FP64 solve's error against the FOM) and
the decoded states after a solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.autoencoder import decode
from oracle.burgers import solve_fom
from oracle.pack import load_pack
from oracle.rom import SQPOptions, evaluate, relative_error, sqp_solve, sqp_step


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module", params=["tinysrpc2x1", "tinysrpc3x1"])
def case(request, dr):
    pack = request.getfixturevalue(request.param + "_pack")
    print(f"[srpc case {request.param}]", flush=True)
    return request.param, pack, dr.Model(pack), load_pack(pack)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def test_srpc_sizes(case):
    name, pack, gm, om = case
    assert gm.n_D == om.n_D and gm.n_C == om.n_C
    for i, (a, b) in enumerate(om.sizes()):
        assert gm.n_om[i] == a and gm.n_ga[i] == b


@pytest.mark.parametrize("B", [1, 70])
def test_srpc_interface_decoders(dr, case, B):
    """Interface rows (every one) and their Jacobians from the port decoders."""
    name, pack, gm, om = case
    ws = dr.Workspace(gm, B)
    for i in range(gm.n_sub):
        dec = om.dec_ga[i]
        xh = si.normal((B, dec.n), seed=700 + i, scale=1.5)
        x, J = (t.cpu().numpy() for t in dr.ae_jacobian_hr(gm, ws, i, 1, xh, precision=dr.PREC_FP64))
        x32, J32 = (t.cpu().numpy() for t in dr.ae_jacobian_hr(gm, ws, i, 1, xh, precision=dr.PREC_FP32_DECODER))
        for b in range(B):
            g, Jr = dec.decode_jacobian(xh[b])
            assert relerr(x[b], g) <= 1e-13 and relerr(J[b], Jr) <= 1e-12
            assert relerr(x32[b], g) <= 2e-6 and relerr(J32[b], Jr) <= 2e-5


def test_srpc_gn_blocks_and_constraint(dr, case):
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
            assert np.array_equal(EG[b, i, :, :m], ev.EG[i])          # the constant Ahat_i, exactly
        assert relerr(c[b], ev.c) <= 1e-13
        assert relerr(rr[b], sum(float(z @ z) for z in ev.Zr)) <= 1e-11


def test_srpc_sqp_step(dr, case):
    name, pack, gm, om = case
    B = 4
    mus = si.heldout_mu(B, 13)
    xh = si.normal((B, gm.n_D), seed=4, scale=0.2)
    lam = si.normal((B, gm.n_C), seed=5, scale=0.01)
    ws = dr.Workspace(gm, B)
    x1, l1, fn, st = (t.cpu().numpy() for t in dr.sqp_step(gm, ws, mus, xh, lam, dr.opts(precision=dr.PREC_FP64)))
    for b in range(B):
        xr, lr, ev, fr, sr, _, alpha = sqp_step(om, mus[b], xh[b], lam[b], SQPOptions())
        print(name, b, "step x err %.2e lam err %.2e alpha %g" % (relerr(x1[b], xr), relerr(l1[b], lr), alpha),
              flush=True)
        assert int(st[b]) == (1 if sr == -1 else sr)
        assert relerr(x1[b], xr) <= 1e-10
        assert relerr(l1[b], lr) <= 1e-8
        assert abs(fn[b] - fr) <= 1e-10 * max(1.0, fr)


@pytest.mark.parametrize("B", [1, 5])
def test_srpc_solve(dr, case, B):
    name, pack, gm, om = case
    mus = si.heldout_mu(B, 17)
    ws = dr.Workspace(gm, B)
    out = {k: v.cpu().numpy() for k, v in dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=100, tol_rel=1e-12,
                                                                                  precision=dr.PREC_FP64)).items()}
    for b in range(B):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-12))
        print(name, b, "status", out["status"][b], ref.status, "iters", out["iters"][b], ref.iters,
              "x err %.2e lam err %.2e" % (relerr(out["xhat"][b], ref.xhat), relerr(out["lam"][b][:gm.n_C], ref.lam)),
              flush=True)
        assert int(out["status"][b]) == ref.status
        assert int(out["iters"][b]) == ref.iters
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        assert relerr(out["lam"][b][:gm.n_C], ref.lam) <= 1e-8
        # the strong constraint holds at the solution
        ev = evaluate(om, mus[b], out["xhat"][b])
        assert np.max(np.abs(ev.c)) <= 1e-12 * max(1.0, np.max(np.abs(out["xhat"][b])))


def test_srpc_fp32_solve_and_states(dr, case):
    """FP32 decoders: error against the FOM within 10% (plus 1e-4) of the FP64 solve's; the decoded
    states (full interior and interface decoders) against the oracle's decoders."""
    name, pack, gm, om = case
    B = 3
    mus = si.heldout_mu(B, 29)
    ws = dr.Workspace(gm, B)
    x64 = dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=60, tol_rel=1e-8, precision=dr.PREC_FP64))["xhat"]
    x32 = dr.rom_solve_batch(gm, ws, mus, dr.opts(max_iter=60, tol_rel=1e-6, precision=dr.PREC_FP32_DECODER,
                                                  stall_tol=1e-5))["xhat"]
    st = dr.decode_states(gm, ws, x64, precision=dr.PREC_FP64).cpu().numpy()
    x64, x32 = x64.cpu().numpy(), x32.cpu().numpy()
    for b in range(B):
        xf = solve_fom(om.fom, mus[b]).x
        e64, e32 = relative_error(om, x64[b], xf), relative_error(om, x32[b], xf)
        print(name, b, "rel err fp64 %.3e fp32 %.3e" % (e64, e32), flush=True)
        assert e32 <= 1.1 * e64 + 1e-4
        off = 0
        for i, (xo, xg) in enumerate(om.split(x64[b])):
            go, gg = decode(om.dec_om[i], xo), om.dec_ga[i].decode(xg)
            n1, n2 = len(go), len(gg)
            assert relerr(st[b, off:off + n1], go) <= 1e-12
            assert relerr(st[b, off + n1:off + n1 + n2], gg) <= 1e-12
            off += n1 + n2
