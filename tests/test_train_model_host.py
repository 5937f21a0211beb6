"""Host-side export of GPU-trained autoencoders (the weights the GPU trainer returns, turned into
the decoders the online solve reads) against the oracle's autoencoder on identical weights:
unpacking, encoding, full decoding and the exported decoder with the de-normalisation folded in
and the latent origin moved.  No GPU is needed: the packed layout is the trainer's."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.autoencoder import ACT_SIGMOID, ACT_SWISH, MaskedAE, Normalisation, decode_jacobian, export_decoder
from paper_2305_15163_amd import ddrom as dr
from paper_2305_15163_amd import train_model as tm


@pytest.mark.parametrize("N,n,b,s,act", [(60, 4, 3, 2, ACT_SIGMOID), (47, 6, 5, 5, ACT_SWISH)])
def test_export_matches_oracle(N, n, b, s, act):
    ae = MaskedAE(N, n, b, s, act)
    p = ae.init_params(3)
    g = si.rng(4)
    p.b1e[:] = g.uniform(-0.3, 0.3, size=p.b1e.shape)
    p.b1d[:] = g.uniform(-0.3, 0.3, size=p.b1d.shape)
    packed = dr.ae_pack(N, n, b, s, *p.as_list()).astype(np.float64)
    # the oracle on the same (FP32-rounded) weights
    q = dr.ae_unpack(packed, N, n, b, s)
    from oracle.autoencoder import AEParams
    pr = AEParams(*[np.asarray(v, dtype=np.float64) for v in q])
    wts = tm.unpack_weights(packed, N, n, b, s)
    Xn = g.uniform(-1, 1, size=(7, N))
    z_ref = ae.encode(pr, Xn)
    z = tm.encode(wts, Xn, N * s, act)
    assert np.max(np.abs(z - z_ref)) <= 1e-12 * max(1.0, np.max(np.abs(z_ref)))
    Y = tm.decode_full(wts, z, N, b, s, act)
    zd = z @ pr.W1d.T + pr.b1d
    from oracle.autoencoder import act as act_fn
    ad, _ = act_fn(zd, act)
    Y_ref = (ae._dec_mat(pr) @ ad.T).T
    assert np.max(np.abs(Y - Y_ref)) <= 1e-12 * max(1.0, np.max(np.abs(Y_ref)))
    # exported decoder == the oracle's export of the same weights, normalisation and centre
    mid, sc = g.normal(size=N), g.uniform(0.5, 2.0, size=N)
    center = z.mean(axis=0)
    dec = tm.export_decoder(wts, mid, sc, center, b, s)
    ref = export_decoder(ae, pr, Normalisation(mid, sc), center)
    assert np.allclose(dec["W1"], ref.W1, rtol=0, atol=0)
    assert np.max(np.abs(dec["b1"] - ref.b1)) <= 1e-13
    assert np.max(np.abs(dec["W2"] - ref.W2vals)) <= 1e-15 * np.max(np.abs(ref.W2vals)) + 0.0
    assert np.array_equal(dec["xref"], ref.x_ref)
    # and it decodes the raw state of the centred latent
    x0, _ = decode_jacobian(ref, np.zeros(n))
    assert np.max(np.abs(x0 - (tm.decode_full(wts, center[None], N, b, s, act)[0] * sc + mid))) <= 1e-12 * np.max(np.abs(x0))


def test_subset_every_keeps_coarse_grid(tmp_path):
    """--subset-to with --every 2: the snapshots of the coarser tensor grid (both grid indices
    even) and the tagged autoencoders' columns, in FP32, with the index lists renumbered."""
    mus = si.training_grid(4, 4)
    X = np.arange(16 * 10, dtype=np.float64).reshape(16, 10) / 7.0
    stem, xs = str(tmp_path / "m"), str(tmp_path / "s_X")
    np.save(xs + ".npy", X)
    np.savez(xs + "_dd.npz", mus=mus)
    np.savez(stem + "_X_dd.npz", om0=np.array([7, 2, 5]), ga0=np.array([5, 9]), om1=np.array([0, 1]))
    np.savez(stem + "_skel.npz", n_sub=np.array(2))
    rows = tm.grid_rows(mus, 2)
    a_vals, l_vals = np.unique(mus[:, 0]), np.unique(mus[:, 1])
    want = [k for k in range(16) if list(a_vals).index(mus[k, 0]) % 2 == 0
            and list(l_vals).index(mus[k, 1]) % 2 == 0]
    assert list(rows) == want and len(rows) == 4
    n = tm.subset_data(stem, ["om0", "ga0"], str(tmp_path / "p"), xs + ".npy", every=2)
    assert n == 4
    Xp = np.load(str(tmp_path / "p_X.npy"))
    dd = np.load(str(tmp_path / "p_X_dd.npz"))
    assert Xp.dtype == np.float32 and Xp.shape == (4, 4)
    for t in ("om0", "ga0"):
        assert np.array_equal(Xp[:, dd[t]], X[rows][:, np.load(stem + "_X_dd.npz")[t]].astype(np.float32))


def test_raw_decoder_round_trip(tmp_path):
    """A raw part (FP32 decoder weights, FP64 normalisation and centre) merged with its skeleton
    gives the pack export_decoder writes, bit for bit."""
    N, n, b, s = 40, 4, 3, 2
    ae = MaskedAE(N, n, b, s, ACT_SIGMOID)
    p = ae.init_params(9)
    packed = dr.ae_pack(N, n, b, s, *p.as_list()).astype(np.float32).astype(np.float64)
    wts = tm.unpack_weights(packed, N, n, b, s)
    g = si.rng(11)
    mid, sc, center = g.normal(size=N), g.uniform(0.5, 2.0, size=N), g.normal(size=n)
    full = tm.export_decoder(wts, mid, sc, center, b, s)
    raw = tm.raw_decoder(wts, mid, sc, center, b, s)
    assert raw["W2"].dtype == np.float32 and raw["W1"].dtype == np.float32
    part = str(tmp_path / "part.npz")
    np.savez(part, **{f"om3_raw_{k}": v for k, v in raw.items()})
    np.savez(str(tmp_path / "m_skel.npz"), n_sub=np.array(4), train_seed=np.array(1))
    out = str(tmp_path / "pack.npz")
    pack = tm.merge([part], out, skeleton=str(tmp_path / "m"))
    assert "train_seed" not in pack and int(pack["n_sub"]) == 4
    for k, v in full.items():
        assert np.array_equal(pack[f"om3_{k}"], v), k
    with pytest.raises(ValueError):
        tm.merge([part], out)
