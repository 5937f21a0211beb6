"""GPU autoencoder training (BF16 matrix-core products, FP32 accumulation and master weights)
against the FP64 oracle: loss and gradient of a minibatch from identical weights, Adam steps,
and a training run against the CPU-trained autoencoder from the same initial weights and
minibatch order.  BF16 operands carry 8 significant bits (relative rounding 2^-9), so the
gradients agree to about 1e-2 in norm; stated per test."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import seeded_inputs as si
from oracle.autoencoder import ACT_SIGMOID, ACT_SWISH, Adam, AEParams, MaskedAE


@pytest.fixture(scope="module")
def dr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_15163_amd as d
    d.lib()
    return d


def _params32(ae, seed):
    p = ae.init_params(seed)
    g = si.rng(seed + 1)
    p.b1e[:] = g.uniform(-0.2, 0.2, size=p.b1e.shape)
    p.b1d[:] = g.uniform(-0.2, 0.2, size=p.b1d.shape)
    # the trainer holds FP32 masters: compare from FP32-representable weights
    return AEParams(*[np.asarray(x, dtype=np.float32).astype(np.float64) for x in p.as_list()])


def _snapshots(N, n_snap, seed):
    """Normalised snapshots in [-1, 1]: a smooth part plus independent noise per component,
    so that an index mixed up with a neighbour's changes the result."""
    g = si.rng(seed)
    x = np.linspace(0.0, 1.0, N)
    X = 0.5 * g.uniform(-1, 1, size=(n_snap, N))
    for k in range(1, 5):
        X += g.normal(size=(n_snap, 1)) / k * np.sin(np.pi * k * x[None, :] + g.uniform(0, 6.3, size=(n_snap, 1)))
    return X / np.max(np.abs(X))


def norm_err(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(1e-30, np.linalg.norm(b)))


@pytest.mark.parametrize("N,n,b,s,act,B", [(150, 4, 3, 2, ACT_SIGMOID, 24), (578, 6, 5, 3, ACT_SIGMOID, 4),
                                           (97, 8, 9, 2, ACT_SWISH, 33)])
def test_ae_loss_and_gradient_parity(dr, N, n, b, s, act, B):
    print(f"[ae grad N={N} n={n} b={b} s={s} act={act} B={B}]", flush=True)
    ae = MaskedAE(N, n, b, s, act)
    p = _params32(ae, 7)
    X = _snapshots(N, B + 9, 8)
    rows = si.rng(9).permutation(B + 9)[:B].astype(np.int32)
    scale = si.rng(10).uniform(0.5, 2.0, size=N)
    ref_loss, ref_g = ae.forward_backward(p, X[rows], scale)
    tr = dr.AETrainer(N, n, b, s, act, B, dr.ae_pack(N, n, b, s, *p.as_list()))
    lt, gt = tr.step(torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda"),
                     torch.as_tensor(rows, device="cuda"),
                     torch.as_tensor(scale.astype(np.float32), device="cuda"), update=False, loss=True, grad=True)
    assert abs(float(lt.item()) - ref_loss) <= 1e-2 * ref_loss
    got = dr.ae_unpack(gt.cpu().numpy(), N, n, b, s)
    names = ["W1e", "b1e", "W2e", "W1d", "b1d", "W2d"]
    errs = {nm: norm_err(gv, rv) for nm, gv, rv in zip(names, got, ref_g.as_list())}
    print("  gradient norm errors", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for nm, e in errs.items():
        assert e < 3e-2, nm


@pytest.mark.parametrize("N,n,b,s,act,B", [(150, 4, 3, 2, ACT_SIGMOID, 24), (97, 8, 9, 2, ACT_SWISH, 33),
                                           (1912, 4, 9, 2, ACT_SIGMOID, 64), (28322, 8, 9, 2, ACT_SIGMOID, 64)])
def test_ae_gradient_elementwise_split_bf16(dr, N, n, b, s, act, B):
    """Split-BF16 mode (each operand as a BF16 head and tail, three matrix-core products:
    about 16 significant bits, FP32 accumulation), every gradient entry against the FP64
    oracle from identical FP32 weights.  The 28322-row case is the largest 120 x 120 subdomain
    of the 480 x 480, 4 x 4 split (the skinny products over w = 56644 then run in 256 split-K
    parts).  Bound per entry: 5e-5 of the tensor's largest entry, about three units of the 2^-16
    left by each split product (sums of up to w terms, activations in FP32; measured 2e-6 to
    1.1e-5); an entry in the wrong band slot, a transposed operand or a dropped term is off by
    the size of the entries themselves."""
    print(f"[ae grad split-bf16 N={N} n={n} b={b} s={s} act={act} B={B}]", flush=True)
    ae = MaskedAE(N, n, b, s, act)
    p = _params32(ae, 17)
    X = _snapshots(N, B + 9, 18)
    rows = si.rng(19).permutation(B + 9)[:B].astype(np.int32)
    scale = si.rng(20).uniform(0.5, 2.0, size=N)
    ref_loss, ref_g = ae.forward_backward(p, X[rows], scale)
    tr = dr.AETrainer(N, n, b, s, act, B, dr.ae_pack(N, n, b, s, *p.as_list()), precision=1)
    lt, gt = tr.step(torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda"),
                     torch.as_tensor(rows, device="cuda"),
                     torch.as_tensor(scale.astype(np.float32), device="cuda"), update=False, loss=True, grad=True)
    lerr = abs(float(lt.item()) - ref_loss) / ref_loss
    got = dr.ae_unpack(gt.cpu().numpy(), N, n, b, s)
    names = ["W1e", "b1e", "W2e", "W1d", "b1d", "W2d"]
    errs = {nm: float(np.max(np.abs(gv - rv)) / max(1e-300, np.max(np.abs(rv))))
            for nm, gv, rv in zip(names, got, ref_g.as_list())}
    print(f"  loss rel err {lerr:.1e}; gradient max entry errors / max entry",
          {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert lerr <= 1e-5
    for nm, e in errs.items():
        assert e <= 5e-5, nm


def test_ae_adam_steps_parity(dr):
    N, n, b, s, B = 120, 4, 3, 2, 16
    ae = MaskedAE(N, n, b, s, ACT_SIGMOID)
    p = _params32(ae, 11)
    X = _snapshots(N, 40, 12)
    scale = np.ones(N)
    tr = dr.AETrainer(N, n, b, s, ACT_SIGMOID, B, dr.ae_pack(N, n, b, s, *p.as_list()))
    opt = Adam(p.as_list(), lr=1e-3)
    Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda")
    sd = torch.as_tensor(scale.astype(np.float32), device="cuda")
    start = [x.copy() for x in p.as_list()]
    for k in range(4):
        rows = si.rng(20 + k).permutation(40)[:B].astype(np.int32)
        tr.step(Xd, torch.as_tensor(rows, device="cuda"), sd, lr=1e-3)
        _, gr = ae.forward_backward(p, X[rows], scale)
        opt.step(p.as_list(), gr.as_list())
    got = dr.ae_unpack(tr.params().cpu().numpy(), N, n, b, s)
    for gv, rv, st in zip(got, p.as_list(), start):
        moved = np.abs(rv - st)
        d = np.abs(gv - rv)
        # every entry moved by up to 4 lr; entries whose gradient sign differs under BF16 may
        # step the other way, the rest agree to a small fraction of a step
        assert np.mean(d < 2e-4) > 0.98 and np.max(d) <= 8.1e-3
        assert np.max(moved) > 1e-3


def test_ae_training_against_cpu(dr, cfg0_pack):
    """The interior autoencoder of subdomain 0 of the 36x36 workload, trained on its 25 FOM
    snapshots for 120 epochs from the oracle's initial weights and minibatch order: the GPU
    (BF16) run reaches a held-out loss close to the CPU (FP64) run's."""
    from oracle.build_model import CONFIGS, snapshots
    from oracle.autoencoder import train as cpu_train
    from oracle.burgers import Grid
    from oracle.ddmaps import build_dd
    from paper_2305_15163_amd.train_ae import train_ae
    cfg = CONFIGS["cfg0"]
    g = Grid(cfg["nx"], cfg["ny"])
    dd = build_dd(g, cfg["nsx"], cfg["nsy"])
    X, _ = snapshots(g.nx, g.ny, si.training_grid(*cfg["train_grid"]), workers=1)
    Xo = X[:, dd.subdomains[0].omega]      # column selection: a Fortran-ordered array
    N, n, b, s = Xo.shape[1], cfg["n_om"], cfg["b"], cfg["s"]
    ae = MaskedAE(N, n, b, s, cfg["act"])
    epochs, seed = 120, 5
    _, _, rep = cpu_train(ae, Xo, seed, epochs, batch=cfg["batch"])
    # the oracle draws its initial weights from the same stream position
    gq = si.rng(seed)
    gq.permutation(Xo.shape[0])
    init = ae.init_params(int(gq.integers(0, 2 ** 62)))
    res = train_ae(Xo, n, b, s, cfg["act"], seed, epochs, batch=cfg["batch"],
                   init=dr.ae_pack(N, n, b, s, *init.as_list()))
    first = res.history[0][1]
    print(f"[ae training] CPU best held-out {rep.test_loss:.4e}, GPU best held-out {res.best_test:.4e} "
          f"(initial {first:.3e})", flush=True)
    assert res.best_test < 0.2 * first
    assert res.best_test <= 1.5 * rep.test_loss


def test_ae_step_rejects_strided_input(dr):
    """A strided tensor would be read with the wrong layout: the binding refuses it."""
    N, n, b, s = 40, 2, 3, 2
    ae = MaskedAE(N, n, b, s, ACT_SIGMOID)
    tr = dr.AETrainer(N, n, b, s, ACT_SIGMOID, 4, dr.ae_pack(N, n, b, s, *_params32(ae, 1).as_list()))
    X = torch.zeros((N, 10), dtype=torch.float32, device="cuda").t()      # [10][N], not contiguous
    with pytest.raises(ValueError):
        tr.step(X, torch.zeros(4, dtype=torch.int32, device="cuda"), torch.ones(N, device="cuda"))
