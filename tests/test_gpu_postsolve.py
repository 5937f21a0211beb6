"""Decoded states and the relative error against the FOM (after a solve) on the GPU,
through the C ABI, against the FP64 oracle's full decoders and its eq. relative_error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.autoencoder import decode
from oracle.burgers import solve_fom
from oracle.pack import load_pack
from oracle.rom import relative_error


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


@pytest.fixture(scope="module", params=["tiny", "cfg0", "tinymix"])
def case(request, dr):
    pack = request.getfixturevalue(request.param + "_pack")
    print(f"[case {request.param}]", flush=True)
    return dr.Model(pack), load_pack(pack)


def oracle_states(om, xhat):
    return np.stack([np.concatenate([np.concatenate([decode(om.dec_om[i], xo), decode(om.dec_ga[i], xg)])
                                     for i, (xo, xg) in enumerate(om.split(x))]) for x in xhat])


@pytest.mark.parametrize("B", [1, 70])
def test_decoded_states_parity(dr, case, B):
    gm, om = case
    xh = si.normal((B, gm.n_D), seed=300 + B, scale=1.0)
    ref = oracle_states(om, xh)
    ws = dr.Workspace(gm, B)
    x64 = dr.decode_states(gm, ws, xh, precision=dr.PREC_FP64).cpu().numpy()
    assert x64.shape == ref.shape
    assert np.max(np.abs(x64 - ref)) <= 1e-12 * np.max(np.abs(ref))
    x32 = dr.decode_states(gm, ws, xh, precision=dr.PREC_FP32_DECODER).cpu().numpy()
    # FP32: a 27-term band sum of weights ~1 and activations in (0, 1), relative ~1e-6
    assert np.max(np.abs(x32 - ref)) <= 2e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("B", [1, 37])
def test_relative_error_parity(dr, case, B):
    gm, om = case
    mus = si.heldout_mu(2, 11)
    fom = [solve_fom(om.fom, m).x for m in mus]
    xf = np.stack([fom[b % 2] * (1.0 + 0.01 * b) for b in range(B)])      # states of several scales
    xh = si.normal((B, gm.n_D), seed=400 + B, scale=0.7)
    ref = np.array([relative_error(om, xh[b], xf[b]) for b in range(B)])
    ws = dr.Workspace(gm, B)
    e64 = dr.relative_error(gm, ws, xh, xf, precision=dr.PREC_FP64).cpu().numpy()
    assert np.max(np.abs(e64 - ref) / ref) <= 1e-12
    e32 = dr.relative_error(gm, ws, xh, xf, precision=dr.PREC_FP32_DECODER).cpu().numpy()
    assert np.max(np.abs(e32 - ref) / ref) <= 1e-4


def test_relative_error_with_exact_subdomain(dr, case):
    """A FOM state that equals subdomain 0's decoded state on its DoFs (ones elsewhere): the
    error has no subdomain-0 term, and the GPU value matches the oracle's."""
    gm, om = case
    xh = si.normal((3, gm.n_D), seed=500, scale=0.5)
    ws = dr.Workspace(gm, 3)
    states = dr.decode_states(gm, ws, xh).cpu().numpy()
    sd0 = om.dd.subdomains[0]
    No, Ng = len(sd0.omega), len(sd0.gamma)
    xf = np.ones((3, gm.N_x))
    xf[:, sd0.omega] = oracle_states(om, xh)[:, :No]
    xf[:, sd0.gamma] = oracle_states(om, xh)[:, No:No + Ng]
    sel = xf[:, np.concatenate([sd0.omega, sd0.gamma])]
    assert np.max(np.abs(states[:, :No + Ng] - sel)) <= 1e-12 * max(1.0, np.max(np.abs(sel)))
    e = dr.relative_error(gm, ws, xh, xf).cpu().numpy()
    ref = np.array([relative_error(om, xh[b], xf[b]) for b in range(3)])
    assert np.max(np.abs(e - ref) / ref) <= 1e-12
