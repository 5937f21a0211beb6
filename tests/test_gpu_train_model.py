"""GPU-trained model packs: every subdomain autoencoder of a skeleton (oracle-written: grid,
split, HR nodes, C, recipe and snapshots, no decoders) trained on the GPU and exported.  The
exported decoders, run by the library's decoder kernel, reproduce the host evaluation of the
trained weights (de-normalisation folded in, latent origin moved), and the model solves."""
import os

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


@pytest.fixture(scope="module")
def trained(dr, tmp_path_factory):
    from oracle.build_model import build
    from oracle.burgers import Grid
    from oracle.ddmaps import build_dd
    from paper_2305_15163_amd.train_model import train_model
    d = tmp_path_factory.mktemp("skel")
    stem = str(d / "tinywide")
    pack, X, mus, _ = build("tinywide", workers=1, verbose=False, train=False)
    np.savez(stem + "_skel.npz", **pack)
    np.save(stem + "_X.npy", X)
    dd = build_dd(Grid(int(pack["nx"]), int(pack["ny"])), int(pack["nsx"]), int(pack["nsy"]))
    idx = {"mus": mus}
    for i, sd in enumerate(dd.subdomains):
        idx[f"om{i}"] = np.asarray(sd.omega, dtype=np.int64)
        idx[f"ga{i}"] = np.asarray(sd.gamma, dtype=np.int64)
    np.savez(stem + "_X_dd.npz", **idx)
    print("[train_model tinywide, 40 epochs, one process]", flush=True)
    out, reports, _ = train_model(stem, procs=1, epochs=40, verbose=False)
    return out, reports


def test_exported_decoders_run_on_the_library(dr, trained):
    from paper_2305_15163_amd.train_model import ACT_SWISH
    pack, reports = trained
    assert len(reports) == 2 * int(pack["n_sub"])
    m = dr.Model(pack)
    B = 5
    ws = dr.Workspace(m, B)
    for i in range(m.n_sub):
        for part, pre in ((0, "om"), (1, "ga")):
            W1, b1 = np.asarray(pack[f"{pre}{i}_W1"]), np.asarray(pack[f"{pre}{i}_b1"])
            W2, xref = np.asarray(pack[f"{pre}{i}_W2"]), np.asarray(pack[f"{pre}{i}_xref"])
            b, s = (int(v) for v in pack[f"{pre}{i}_bs"])
            N, n = xref.shape[0], W1.shape[1]
            xh = si.normal((B, n), seed=40 + 2 * i + part, scale=0.7)
            z = xh @ W1.T + b1
            a = z / (1.0 + np.exp(-z))                      # Swish
            full = np.tile(xref, (B, 1))
            for k in range(3):
                for t in range(b):
                    c = np.arange(N) * s + (k - 1) * b * s + t
                    ok = (c >= 0) & (c < W1.shape[0])
                    full[:, ok] += a[:, c[ok]] * W2[ok, k, t]
            rows = m.subnet_rows(i, part)
            got = dr.ae_decode_hr(m, ws, i, part, xh, precision=dr.PREC_FP64).cpu().numpy()
            assert np.max(np.abs(got - full[:, rows])) <= 1e-12 * max(1.0, np.max(np.abs(full)))
    assert int(pack["act"]) == ACT_SWISH


def test_gpu_trained_model_solves(dr, trained):
    pack, _ = trained
    m = dr.Model(pack)
    mus = si.heldout_mu(4, 51)
    ws = dr.Workspace(m, len(mus))
    r = dr.rom_solve_batch(m, ws, mus, dr.opts(max_iter=60, tol_rel=1e-8, precision=dr.PREC_FP64))
    st = r["status"].cpu().numpy()
    print("statuses", st.tolist(), "iterations", r["iters"].cpu().tolist(), flush=True)
    assert np.all(np.isfinite(r["xhat"].cpu().numpy())) and np.all(st != 4)
    assert (st == 0).sum() >= len(st) // 2
