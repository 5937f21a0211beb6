"""Parity at the benchmark's own shape: 240 x 240 grid, 4 x 4 subdomains, latents (8, 4),
360 HR nodes per subdomain, 32 constraints (the trained pack the benchmark solves when it is
present, else a pack of the same shape from the oracle pipeline).  Batches span three or more
64-solve groups, so the schedules the benchmark runs are the ones checked: the FP32 decoder's
one-group-per-wave schedule (more than 128 live solves), grids of more than two solve groups,
and the update kernel instantiated for 12-entry blocks with 4 interface latents.  The oracle
computes sampled lanes one by one (FP64 throughout)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.autoencoder import decode_jacobian
from oracle.pack import load_pack
from oracle.rom import SQPOptions, evaluate, kkt_matrix, sqp_solve, sqp_step

LANES = (0, 1, 63, 64, 127, 128, 190, 191)     # first, second, group edges and the ragged tail of B = 192


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module")
def head(dr, headline_pack):
    name, pack = headline_pack
    print(f"[headline pack {name}]", flush=True)
    gm, om = dr.Model(pack), load_pack(pack)
    assert gm.n_sub == 16 and gm.n_C == 32 and gm.n_D == 192
    assert all(a == 8 and b == 4 for a, b in om.sizes())
    assert all(gm.size(16, i) == 360 for i in range(16))
    return name, gm, om


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def test_headline_decoders_fp32_wide_batch(dr, head):
    """FP32 interior subnets and interface decoders at B = 192 (every row, sampled lanes)
    against the FP64 oracle's full decoders, within FP32 rounding of the 27-term band sums."""
    name, gm, om = head
    B = 192
    ws = dr.Workspace(gm, B)
    for i in (0, 5, 15):
        for part, dec in ((0, om.dec_om[i]), (1, om.dec_ga[i])):
            print(f"[headline fp32 decoder sd {i} part {part}]", flush=True)
            rows = gm.subnet_rows(i, part)
            xh = si.normal((B, dec.n), seed=300 + 3 * i + part, scale=1.0)
            x, J = (t.cpu().numpy() for t in dr.ae_jacobian_hr(gm, ws, i, part, xh, precision=dr.PREC_FP32_DECODER))
            for b in LANES:
                g, Jr = decode_jacobian(dec, xh[b])
                assert relerr(x[b], g[rows]) <= 2e-6
                assert relerr(J[b], Jr[rows]) <= 2e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_headline_gn_blocks(dr, head, precision):
    """H_i, g_i, C A_i dg_i^Gamma/dxhat, the constraint and sum ||Z r_i||^2 at B = 192.  FP64:
    1e-11 / 1e-10 / 1e-12 as at the small sizes; FP32 decoders: 1e-4 (FP32 rounding of decoder
    values and Jacobians carried through the FP64 residual, about 1e-6 relative per entry)."""
    name, gm, om = head
    print(f"[headline gn blocks precision={precision}]", flush=True)
    B = 192
    mus = si.heldout_mu(B, 61)
    xh = si.normal((B, gm.n_D), seed=62, scale=0.5)
    ws = dr.Workspace(gm, B)
    H, g, EG, c, rr = (t.cpu().numpy() for t in dr.gn_blocks(gm, ws, mus, xh, precision=precision))
    tH, tg, tE = (1e-11, 1e-10, 1e-12) if precision == 0 else (1e-4, 1e-4, 1e-4)
    for b in LANES:
        ev = evaluate(om, mus[b], xh[b])
        for i, (o, (a, m)) in enumerate(zip(om.offsets(), om.sizes())):
            assert relerr(H[b, i, :a + m, :a + m], ev.H[i]) <= tH
            assert relerr(g[b, o:o + a + m], ev.g[i]) <= tg
            assert relerr(EG[b, i, :, :m], ev.EG[i]) <= tE
        assert relerr(c[b], ev.c) <= tE
        assert relerr(rr[b], sum(float(z @ z) for z in ev.Zr)) <= tH


def test_headline_sqp_step(dr, head):
    """One SQP iteration at B = 192 in FP64 (the 12-entry-block update kernel with a 32 x 32
    Schur complement): sampled lanes against the oracle's step (dense LAPACK KKT solve).
    x and the multiplier to 1e-10."""
    name, gm, om = head
    print("[headline sqp_step]", flush=True)
    B = 192
    mus = si.heldout_mu(B, 63)
    xh = si.normal((B, gm.n_D), seed=64, scale=0.2)
    lam = si.normal((B, gm.n_C), seed=65, scale=0.01)
    ws = dr.Workspace(gm, B)
    x1, l1, fn, st = (t.cpu().numpy() for t in dr.sqp_step(gm, ws, mus, xh, lam, dr.opts(precision=dr.PREC_FP64)))
    for b in LANES[::2]:
        xr, lr, ev, fr, sr, _, _ = sqp_step(om, mus[b], xh[b], lam[b], SQPOptions())
        kap = np.linalg.cond(kkt_matrix(om, evaluate(om, mus[b], xh[b])))
        print(f"  lane {b}: x err {relerr(x1[b], xr):.2e} lam err {relerr(l1[b], lr):.2e} cond(K) {kap:.2e}",
              flush=True)
        assert int(st[b]) == (1 if sr == -1 else sr)
        assert relerr(x1[b], xr) <= 1e-10
        assert relerr(l1[b], lr) <= 1e-10
        assert abs(fn[b] - fr) <= 1e-10 * max(1.0, fr)


def test_headline_fp64_solves(dr, head):
    """Full FP64 solves from the zero start at B = 160 (three solve groups, the last ragged);
    eight sampled parameters against the oracle's solves: same status, same iteration count,
    xhat to 1e-10 where the solve converged.  A solve that stops on a failure (possible with the
    briefly trained stand-in pack, whose decoders let some solves drift until a block or the
    Schur complement loses definiteness) is compared to max(1e-10, 100 cond(K) eps) with K the
    KKT matrix at the oracle's stopping point."""
    name, gm, om = head
    print("[headline fp64 solves]", flush=True)
    B = 160
    mus = si.heldout_mu(B, 1)
    ws = dr.Workspace(gm, B)
    o = dr.opts(max_iter=60, tol_rel=1e-10, precision=dr.PREC_FP64)
    out = {k: v.cpu().numpy() for k, v in dr.rom_solve_batch(gm, ws, mus, o).items()}
    for b in (0, 1, 63, 64, 100, 127, 128, 159):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=60, tol_abs=0.0, tol_rel=1e-10))
        print(f"  mu {b}: status gpu {int(out['status'][b])} oracle {ref.status}, iters gpu {int(out['iters'][b])} "
              f"oracle {ref.iters}, x err {relerr(out['xhat'][b], ref.xhat):.2e}", flush=True)
        assert int(out["status"][b]) == ref.status
        assert int(out["iters"][b]) == ref.iters
        tol = 1e-10
        if ref.status != 0:
            kap = np.linalg.cond(kkt_matrix(om, evaluate(om, mus[b], ref.xhat)))
            tol = max(tol, 100 * kap * np.finfo(float).eps)
        assert relerr(out["xhat"][b], ref.xhat) <= tol
        assert abs(out["fnorm0"][b] - ref.fnorm0) <= 1e-12 * ref.fnorm0
