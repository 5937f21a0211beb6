"""The allocation-free decoder entry point (ae_jacobian_hr_noalloc, staging in the library's
static device array) against ae_jacobian_hr with a workspace: same kernels and arithmetic, so
values and Jacobians must agree bitwise; two calls in a row per decoder, the second with a
smaller batch (the array keeps the first call's contents), and a batch beyond the array's
size rejected before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.mark.parametrize("name", ["tiny", "cfg0"])
@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_workspace_entry(dr, request, name, precision):
    pack = request.getfixturevalue(name + "_pack")
    gm = dr.Model(pack)
    ws = dr.Workspace(gm, 130)
    dt = torch.float64 if precision == 0 else torch.float32
    for B in (130, 7):          # three 64-solve groups (ragged), then a smaller batch
        print(f"[noalloc {name} precision={precision} B={B}]", flush=True)
        for sd in range(gm.n_sub):
            for part in (0, 1):
                n = gm.n_om[sd] if part == 0 else gm.n_ga[sd]
                rows = gm.size(14, sd) if part == 0 else gm.N_ga[sd]
                xh = torch.as_tensor(si.normal((B, n), seed=200 + 11 * sd + part + B, scale=1.5), device="cuda")
                x_ref, J_ref = dr.ae_jacobian_hr(gm, ws, sd, part, xh, precision=precision)
                x = torch.full((B, rows), float("nan"), dtype=dt, device="cuda")
                J = torch.full((B, rows, n), float("nan"), dtype=dt, device="cuda")
                dr.ae_jacobian_hr_noalloc(gm, sd, part, xh, x, J, precision=precision)
                J2 = torch.full((B, rows, n), float("nan"), dtype=dt, device="cuda")
                dr.ae_jacobian_hr_noalloc(gm, sd, part, xh, None, J2, precision=precision)
                torch.cuda.synchronize()
                assert torch.equal(x, x_ref) and torch.equal(J, J_ref) and torch.equal(J2, J_ref)


def test_noalloc_rejects_batch_beyond_scratch(dr, cfg0_pack):
    """cfg0's interior subnet needs rows * 7 * 8 bytes per solve in FP64; 4096 solves exceed
    the 16 MiB array: an error before any launch, and the entry point still works after it."""
    gm = dr.Model(cfg0_pack)
    rows = gm.size(14, 0)
    B = 4096
    assert rows * 7 * B * 8 > 16 << 20
    xh = torch.zeros((B, gm.n_om[0]), dtype=torch.float64, device="cuda")
    J = torch.empty((B, rows, gm.n_om[0]), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="staging"):
        dr.ae_jacobian_hr_noalloc(gm, 0, 0, xh, None, J, precision=0)
    ws = dr.Workspace(gm, 3)
    x_ref, J_ref = dr.ae_jacobian_hr(gm, ws, 0, 0, xh[:3], precision=0)
    J3 = torch.empty((3, rows, gm.n_om[0]), dtype=torch.float64, device="cuda")
    dr.ae_jacobian_hr_noalloc(gm, 0, 0, xh[:3].contiguous(), None, J3, precision=0)
    torch.cuda.synchronize()
    assert torch.equal(J3, J_ref)
