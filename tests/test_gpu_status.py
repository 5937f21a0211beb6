"""Stop statuses of the batched solve on the GPU (through the C ABI) against the FP64 oracle:
KKT_NOT_PD (a singular block H_i; a constraint Jacobian without full row rank, at the start
and inside a step), NONFINITE (NaN parameters inside an otherwise ordinary batch), STALLED
(FP64 run to its rounding floor with the stagnation stop set), LINESEARCH_FAIL (no
backtracking allowed) and the iteration cap max_iter = 1.  The failure constructions make
Lemma 1's hypotheses fail exactly (see status_cases.py), so both sides must agree on them."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.pack import load_pack
from oracle.rom import (KKT_NOT_PD, LINESEARCH_FAIL, MAX_ITER, NONFINITE, STALLED, SQPOptions, evaluate, kkt_rhs,
                        sqp_solve, sqp_step)
from status_cases import rank_deficient_constraint, singular_block


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def _solve(dr, pack, mus, **kw):
    gm = dr.Model(pack)
    ws = dr.Workspace(gm, len(mus))
    out = dr.rom_solve_batch(gm, ws, mus, dr.opts(precision=dr.PREC_FP64, **kw))
    return gm, {k: v.cpu().numpy() for k, v in out.items()}


def test_kkt_not_pd_rank_deficient_constraint(dr, tiny_pack):
    """Zero row of C: the initial multiplier's normal equations are singular; every solve
    stops at the start with KKT_NOT_PD, lambda = 0, ||F(0, 0)||."""
    print("[status kkt_not_pd: rank-deficient constraint]", flush=True)
    pack = rank_deficient_constraint(tiny_pack)
    om = load_pack(pack)
    mus = si.heldout_mu(5, 11)
    gm, out = _solve(dr, pack, mus, max_iter=20, tol_rel=1e-10)
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=20, tol_abs=0.0, tol_rel=1e-10))
        assert ref.status == KKT_NOT_PD
        assert int(out["status"][b]) == KKT_NOT_PD and int(out["iters"][b]) == 0
        assert np.all(out["xhat"][b] == 0.0) and np.all(out["lam"][b][:gm.n_C] == 0.0)
        assert abs(out["fnorm"][b] - ref.fnorm) <= 1e-12 * ref.fnorm


def test_kkt_not_pd_rank_deficient_constraint_step(dr, tiny_pack):
    """The same construction with the multiplier given: the Schur complement of the step is
    singular, sqp_step reports KKT_NOT_PD and leaves the point unchanged."""
    print("[status kkt_not_pd: sqp_step]", flush=True)
    pack = rank_deficient_constraint(tiny_pack)
    om = load_pack(pack)
    gm = dr.Model(pack)
    B = 3
    mus = si.heldout_mu(B, 13)
    xh = si.normal((B, gm.n_D), seed=4, scale=0.2)
    lam = si.normal((B, gm.n_C), seed=5, scale=0.01)
    ws = dr.Workspace(gm, B)
    x1, l1, fn, st = (t.cpu().numpy() for t in dr.sqp_step(gm, ws, mus, xh, lam, dr.opts(precision=dr.PREC_FP64)))
    for b in range(B):
        xr, lr, _, fr, sr, _, _ = sqp_step(om, mus[b], xh[b], lam[b], SQPOptions())
        assert sr == KKT_NOT_PD and int(st[b]) == KKT_NOT_PD
        assert np.array_equal(x1[b], xh[b]) and np.array_equal(l1[b], lam[b])
        assert abs(fn[b] - fr) <= 1e-12 * fr


def test_kkt_not_pd_singular_block(dr, tiny_pack):
    """Zero column of an interior decoder's W1: H_0 has an exactly zero pivot at the first
    step; KKT_NOT_PD at the start point with the least-squares multiplier."""
    print("[status kkt_not_pd: singular block]", flush=True)
    pack = singular_block(tiny_pack, sd=0, col=1)
    om = load_pack(pack)
    mus = si.heldout_mu(4, 11)
    gm, out = _solve(dr, pack, mus, max_iter=20, tol_rel=1e-10)
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=20, tol_abs=0.0, tol_rel=1e-10))
        assert ref.status == KKT_NOT_PD and ref.iters == 0
        assert int(out["status"][b]) == KKT_NOT_PD and int(out["iters"][b]) == 0
        assert np.all(out["xhat"][b] == 0.0)
        assert relerr(out["lam"][b][:gm.n_C], ref.lam) <= 1e-10
        assert abs(out["fnorm"][b] - ref.fnorm) <= 1e-12 * ref.fnorm


def test_nonfinite_parameters_in_a_batch(dr, tiny_pack):
    """NaN parameters stop their own solves with NONFINITE at iteration 0; the other solves of
    the batch are untouched (bitwise equal to a batch without the NaN entries) and match the
    oracle."""
    print("[status nonfinite]", flush=True)
    om = load_pack(tiny_pack)
    mus = si.heldout_mu(6, 31)
    bad = mus.copy()
    bad[1, 0] = np.nan
    bad[4, 1] = np.nan
    kw = dict(max_iter=100, tol_rel=1e-12)
    gm, out = _solve(dr, tiny_pack, bad, **kw)
    _, ref_out = _solve(dr, tiny_pack, mus, **kw)
    for b in range(len(mus)):
        if b in (1, 4):
            ref = sqp_solve(om, bad[b], opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-12))
            assert ref.status == NONFINITE
            assert int(out["status"][b]) == NONFINITE and int(out["iters"][b]) == 0
            assert not np.isfinite(out["fnorm"][b])
        else:
            for k in ("xhat", "lam", "iters", "status", "fnorm"):
                assert np.array_equal(out[k][b], ref_out[k][b]), k
            ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=100, tol_abs=0.0, tol_rel=1e-12))
            assert int(out["status"][b]) == ref.status
            assert relerr(out["xhat"][b], ref.xhat) <= 1e-10


def test_stalled_fp64(dr, tiny_pack):
    """FP64 with an unreachable tolerance and stall_tol = 1e-6: both sides iterate to the
    rounding floor and stop STALLED.  Which iteration first fails the Armijo test there is
    decided by rounding, so the iteration counts may differ; what is unique is the solution
    both reach (compared to 1e-10) and the stop rule itself (checked on the GPU's own
    returned point: ||F|| <= stall_tol ||F_0||)."""
    print("[status stalled fp64]", flush=True)
    om = load_pack(tiny_pack)
    mus = si.heldout_mu(4, 11)
    gm, out = _solve(dr, tiny_pack, mus, max_iter=200, tol_rel=0.0, stall_tol=1e-6)
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=200, tol_abs=0.0, tol_rel=0.0, stall_tol=1e-6))
        print(f"  mu {b}: status gpu {int(out['status'][b])} oracle {ref.status}, iters gpu {int(out['iters'][b])} "
              f"oracle {ref.iters}, |F|/|F0| gpu {out['fnorm'][b] / out['fnorm0'][b]:.2e} oracle "
              f"{ref.fnorm / ref.fnorm0:.2e}", flush=True)
        assert ref.status == STALLED and int(out["status"][b]) == STALLED
        assert out["fnorm"][b] <= 1e-6 * out["fnorm0"][b]
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        # the GPU's stopping point is a valid stop for the oracle's own arithmetic as well
        ev = evaluate(om, mus[b], out["xhat"][b])
        f = np.linalg.norm(kkt_rhs(om, ev, out["lam"][b][:gm.n_C]))
        assert f <= 1e-6 * ref.fnorm0


def test_linesearch_fail_no_backtracking(dr, tiny_pack):
    """max_backtracks = 0: solves whose full KKT step fails the Armijo test stop with
    LINESEARCH_FAIL at the same iteration and point as the oracle's; the others run to the
    iteration cap or converge, also as the oracle's do."""
    print("[status linesearch_fail]", flush=True)
    om = load_pack(tiny_pack)
    mus = si.heldout_mu(8, 17)
    gm, out = _solve(dr, tiny_pack, mus, max_iter=10, tol_rel=1e-12, max_backtracks=0)
    n_fail = 0
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=10, tol_abs=0.0, tol_rel=1e-12, max_backtracks=0))
        print(f"  mu {b}: status gpu {int(out['status'][b])} oracle {ref.status}, iters gpu {int(out['iters'][b])} "
              f"oracle {ref.iters}", flush=True)
        assert int(out["status"][b]) == ref.status and int(out["iters"][b]) == ref.iters
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        n_fail += ref.status == LINESEARCH_FAIL
    assert n_fail >= 2


@pytest.mark.parametrize("name", ["tiny", "cfg0", "tinymix"])
def test_max_iter_one(dr, request, name):
    """max_iter = 1: one accepted step from the zero start, status MAX_ITER, the oracle's
    point to 1e-10."""
    print(f"[status max_iter=1 {name}]", flush=True)
    pack = request.getfixturevalue(name + "_pack")
    om = load_pack(pack)
    mus = si.heldout_mu(5, 19)
    gm, out = _solve(dr, pack, mus, max_iter=1, tol_rel=1e-12)
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=1, tol_abs=0.0, tol_rel=1e-12))
        assert ref.status == MAX_ITER and ref.iters == 1
        assert int(out["status"][b]) == MAX_ITER and int(out["iters"][b]) == 1
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
        assert abs(out["fnorm"][b] - ref.fnorm) <= 1e-10 * ref.fnorm


def test_stall_ratio_fp64(dr, tiny_pack):
    """The progress form of the stagnation stop (stall_ratio) in FP64, where it fires well above
    the rounding floor: the same step, status and point as the oracle's.  The decisive ratio of
    each case is checked to be far from the threshold, so rounding cannot flip the decision."""
    print("[status stall_ratio fp64]", flush=True)
    om = load_pack(tiny_pack)
    mus = si.heldout_mu(3, 11)
    theta, stol = 0.05, 1e-3
    gm, out = _solve(dr, tiny_pack, mus, max_iter=60, tol_rel=1e-14, stall_tol=stol, stall_ratio=theta)
    for b in range(len(mus)):
        ref = sqp_solve(om, mus[b], opts=SQPOptions(max_iter=60, tol_abs=0.0, tol_rel=1e-14, stall_tol=stol,
                                                    stall_ratio=theta))
        h = ref.history
        print(f"  mu {b}: status gpu {int(out['status'][b])} oracle {ref.status}, iters gpu {int(out['iters'][b])} "
              f"oracle {ref.iters}, ratio {h[ref.iters] / h[ref.iters - 1]:.3e}", flush=True)
        assert ref.status == STALLED
        assert abs(h[ref.iters] / h[ref.iters - 1] - theta) > 1e-3 * theta
        assert int(out["status"][b]) == STALLED and int(out["iters"][b]) == ref.iters
        assert relerr(out["xhat"][b], ref.xhat) <= 1e-10
