"""Benchmark: batched HR DD NM-ROM solves/sec on one MI355X.

Workload (default): steady 2D Burgers on a 240x240 interior grid, 4x4 subdomains,
latents (n^Omega, n^Gamma) = (8, 4), decoder width 2x DoFs, three-band mask with b = 9,
HR on 10% of each subdomain's nodes, 512 held-out (a, lambda) drawn uniformly, FP32
decoders with FP64 residual / Gauss-Newton blocks / KKT / line search.  Solves are
warm-started from the learned proposal (2 -> 256 -> 256 -> 224 SiLU network trained on the
method's own solves) with the zero start as fallback.
One step = one rom_solve_warm call over the 512 parameters (proposal inference and all
solver rounds, replayed from a captured HIP graph).  value = solves per second over the
timed steps.  The zero-start batch (rom_solve_batch) is timed the same way beside it.

The model pack (trained decoders, HR nodes, C) is read from models/<config>.npz, which the
offline pipeline writes (python -m oracle.build_model <config>); the proposal from
models/<config>_mlp.npz (python -m paper_2305_15163_amd.train_proposal).  Without the
proposal file the zero-start batch is the headline.

Also reported: the dominant kernel's roofline figures (HIP-event timed launches on the
library's stream), plain per-solve GPU SQP (B = 1, FP64, sequential calls) and the CPU
oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HR DD NM-ROM solves/sec on 1 MI355X vs plain SQP at fixed rel. error vs FOM"
PEAK_FP32_VECTOR_TFLOPS = 157.3   # published FP32 vector peak (packed FP32 issue)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # one FP32 FMA per lane per clock: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM traffic of the interior-decoder timing launch (k_decode<float, 8, 0, 4, 1, 0>, B = 512), from two
# counter runs of `bench.py --roofline-only` (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE; KiB per
# dispatch, mean of 20), each scaled by what the same counter reads for a 256 MiB device copy in the
# same run (FETCH_SIZE 131084.6 KiB, WRITE_SIZE 262144 KiB for 262144 KiB moved).  Valid only for the
# decoder source and work-item shape it was measured on; otherwise traffic is reported as null.
DECODE_COUNTERS = dict(fetch_kib=10856.4, write_kib=288288.0, fetch_scale=262144.0 / 131084.6, write_scale=1.0,
                       source_sha1="c3fd6c4c95e7c205", tile=(16, 24, 256),
                       profile="profiles/k_decode_f32_burgers240_4x4_b512.md")


def decoder_source_sha1():
    """Hash of the decoder kernel's source text and of the ring sizes it is instantiated with."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2305_15163_amd", "csrc", "kernels.hip")) as f:
        s = f.read()
    with open(os.path.join(ROOT, "paper_2305_15163_amd", "csrc", "internal.h")) as f:
        ring = "".join(ln for ln in f if ln.startswith("constexpr int DEC_RING"))
    i = s.index("template <typename T, int NL, int ACT, int WAVES, int TAG, int VO = 0, int RING = DEC_RING>\n__global__")
    j = s.index("\n}\n", i) + 3
    return hashlib.sha1((s[i:j] + ring).encode()).hexdigest()[:16]


CONFIGS = {
    "cfg1": dict(batch=512, seed=1, proposal_seed=5, precision=1, tol_rel=1e-6, stall_tol=1e-5, stall_ratio=0.5,
                 max_iter=60,
                 workload="Burgers 240x240, 4x4 subdomains, latent (8,4), width 2x, band 9, HR 10%, "
                          "512 held-out (a,lambda), FP32 decoder + FP64 KKT"),
    "cfg0": dict(batch=1, seed=0, proposal_seed=5, precision=0, tol_rel=1e-8, stall_tol=0.0, stall_ratio=0.0,
                 max_iter=60,
                 workload="Burgers 36x36, 2x2 subdomains, latent (6,3), width 3x, band 5, HR 20%, "
                          "1 held-out (a,lambda), FP64"),
}


def decoder_work(model, B):
    """Algorithmic FLOPs and bytes of one interior-decoder launch over B solves.
    Per solve and subdomain: 2 n |I_h| (hidden pre-activations) + sum over kept rows of
    q_r (3 + 2 n) (value FMA, sigma' scaling, n Jacobian FMAs per band entry); activations'
    transcendentals are not counted.  Bytes (FP32): subnet weights read once, FP64 latents
    read, value + Jacobian rows written."""
    flops = 0.0
    wbytes = 0.0
    obytes = 0.0
    for i in range(model.n_sub):
        n = model.n_om[i]
        H = model.size(15, i)
        O = model.size(14, i)
        q = model.size(19, i)
        flops += 2.0 * n * H + q * (3.0 + 2.0 * n)
        wbytes += 4.0 * (H * n + H + q + O) + 8.0 * 3 * O
        obytes += 4.0 * O * (1 + n)
    return flops * B, wbytes + B * (obytes + 8.0 * model.n_D)


UNEVEN = dict(models=("cfg2a", "cfg2b", "cfg2c"), batch=1024, seed=2, precision=1, tol_rel=1e-6, stall_tol=1e-5,
              stall_ratio=0.5, n_err=16,
              max_iter=60,
              workload="uneven batch: 1024 held-out (a,lambda) split evenly (seeded) over three Burgers models "
                       "with 60x60-node subdomains: 120x120 2x2, 240x240 4x4, 480x480 8x8; per-subdomain latent "
                       "sizes from {4,6,8,12} and HR fractions from [5%, 25%]; FP32 decoder + FP64 KKT; zero start",
              # autoencoders trained on the GPU on FOM snapshots (models/<model>_gpu.npz) when present,
              # else the CPU-trained packs of the offline pipeline (models/<model>.npz)
              gpu_trained="1024 (120x120) or 256 (240x240, 480x480) FOM snapshots, GPU training to 2000 epochs")


def uneven_leg(a, torch, dr):
    """1024 solves over three models in one multi-model graph (rom_solve_multi), each model with
    the work-item shape of the persisted table (measured by the shape search when missing);
    timed like the headline, and beside it the same solves as three rom_solve_batch calls."""
    from paper_2305_15163_amd import autotune
    import seeded_inputs as si
    cfg = UNEVEN
    gpu = [os.path.join(ROOT, "models", f"{c}_gpu.npz") for c in cfg["models"]]
    trained_on_gpu = all(os.path.exists(p) for p in gpu) and not a.uneven_cpu_packs
    paths = gpu if trained_on_gpu else [os.path.join(ROOT, "models", f"{c}.npz") for c in cfg["models"]]
    missing = [p for p in paths if not os.path.exists(p)]
    if missing:
        print(f"[bench] uneven batch skipped: missing {missing}", file=sys.stderr, flush=True)
        return None
    B = cfg["batch"]
    mu_all = si.heldout_mu(B, cfg["seed"])
    which = si.model_assignment(B, len(paths), cfg["seed"])
    o = dr.opts(max_iter=cfg["max_iter"], tol_rel=cfg["tol_rel"], precision=cfg["precision"], stall_tol=cfg["stall_tol"],
                stall_ratio=cfg["stall_ratio"])
    table = os.path.join(ROOT, "paper_2305_15163_amd", "tiles.json")
    models, wss, mus, tiles, info = [], [], [], [], []
    for k, p in enumerate(paths):
        pack = dict(np.load(p, allow_pickle=False))
        mu_k = np.ascontiguousarray(mu_all[which == k])
        tile = autotune.tiles_for(pack, mu_k, o, path=table, verbose=True)
        m = dr.Model(pack, tile=tile)
        models.append(m)
        wss.append(dr.Workspace(m, len(mu_k)))
        mus.append(torch.as_tensor(mu_k, device="cuda"))
        tiles.append(list(m.tile))
        info.append({"model": cfg["models"][k], "solves": int(len(mu_k)), "subdomains": m.n_sub, "n_D": m.n_D,
                     "n_C": m.n_C, "tile": list(m.tile)})
        del pack
        print(f"[bench] uneven: model {cfg['models'][k]} ready ({len(mu_k)} solves, tile {m.tile})",
              file=sys.stderr, flush=True)

    def run_multi():
        return dr.rom_solve_multi(models, wss, mus, o)

    def run_one(k):
        return lambda: dr.rom_solve_batch(models[k], wss[k], mus[k], o)

    def timed(fn, tag):
        for w in range(a.warmup):
            fn()
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            outs = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench] uneven {tag}: timed {a.steps} steps in {dt:.3f}s", file=sys.stderr, flush=True)
        return dt, outs

    dt_m, outs = timed(run_multi, "multi-model graph")
    # the same solves as one batch per model, one after the other: the sum of these times is what
    # the multi-model solve's concurrency is measured against, the largest is its lower bound
    dt_k = [timed(run_one(k), f"model {cfg['models'][k]} alone")[0] for k in range(len(models))]
    dt_s = sum(dt_k)
    for k, d in enumerate(dt_k):
        info[k]["ms_alone"] = 1e3 * d / a.steps
    for k, r in enumerate(outs):
        st = r["status"].cpu().numpy()
        it = r["iters"].cpu().numpy()
        info[k]["iters_mean"] = float(it.mean())
        info[k]["status_counts"] = {dr.STATUS[s]: int((st == s).sum()) for s in np.unique(st)}
        # error against the FOM (eq. relative_error) on the model's first solves, when the offline
        # reference states of exactly those parameters are stored
        ne = min(cfg["n_err"], len(mus[k]))
        Xf = fom_reference(cfg["models"][k], [("uneven", mus[k][:ne].cpu().numpy())])[0]
        if Xf is not None:
            e = dr.relative_error(models[k], wss[k], r["xhat"][:ne].contiguous(),
                                  torch.as_tensor(Xf, device="cuda")).cpu().numpy()
            info[k]["rel_err_vs_fom"] = error_summary(e, st[:ne], dr)
    stopped_ok = sum(v.get("converged", 0) + v.get("stalled", 0) for v in (i["status_counts"] for i in info))
    converged = sum(i["status_counts"].get("converged", 0) for i in info)
    return {"workload": cfg["workload"], "packs": [os.path.relpath(p, ROOT) for p in paths],
            "autoencoders": ("trained on the GPU: " + cfg["gpu_trained"]) if trained_on_gpu else
                            "trained by the FP64 CPU pipeline (8 x 8 parameter grid, 300 epochs)",
            "solves_per_s": B * a.steps / dt_m, "ms_per_step": 1e3 * dt_m / a.steps,
            "converged_solves_per_s": converged * a.steps / dt_m,
            "converged_or_stalled_solves_per_s": stopped_ok * a.steps / dt_m,
            "separate_batches_solves_per_s": B * a.steps / dt_s, "models": info,
            "tiles_from": "work-item shape search (ddrom_autotune), table paper_2305_15163_amd/tiles.json"}


AE_SHAPES = (("interior", 28322, 8), ("interface", 1912, 4))   # N, latent: the largest 120x120-subdomain AEs


def ae_training_leg(a, torch, dr, si):
    """GPU autoencoder training steps at the 480x480, 4x4 workload's largest subdomain shapes
    (interior N = 28322, latent 8; interface N = 1912, latent 4), width 2N, band 9, minibatch 64,
    BF16 matrix-core products with FP32 accumulation, FP32 masters and Adam.  Synthetic
    snapshots in [-1, 1].  Per step: FLOPs = 2 B (4 nnz + 6 n w) (forward and backward of the two
    band layers and the two dense layers); algorithmic bytes = the minibatch read twice
    (input and target, FP32) + 36 bytes per parameter (BF16 weights read in the forward and
    backward passes: 4; FP32 gradient written and read: 8; Adam's FP32 master, m and v read and
    written: 24)."""
    from paper_2305_15163_amd.train_ae import glorot_init
    B, out = 64, []
    for name, N, n in AE_SHAPES:
        b_, s_ = 9, 2
        tr = dr.AETrainer(N, n, b_, s_, 0, B, glorot_init(N, n, b_, s_, 3))
        X = torch.as_tensor(si.uniform((256, N), -1, 1, 5).astype(np.float32), device="cuda")
        sc = torch.ones(N, device="cuda")
        rows = [torch.as_tensor(si.rng(k).permutation(256)[:B].astype(np.int32), device="cuda") for k in range(8)]
        for k in range(5):
            tr.step(X, rows[k % 8], sc)
        torch.cuda.synchronize()
        K = 50
        t0 = time.perf_counter()
        for k in range(K):
            tr.step(X, rows[k % 8], sc)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        cols, valid = dr.ddrom.band_slots(N, b_, s_)
        nnz, w = int(valid.sum()), N * s_
        n_par = int(tr.n_params)
        flops = 2.0 * B * (4 * nnz + 6 * n * w)
        bytes_ = 2.0 * B * N * 4 + 36.0 * n_par
        out.append({"autoencoder": name, "N": N, "latent": n, "width": w, "parameters": n_par, "batch": B,
                    "ms_per_step": 1e3 * dt, "samples_per_s": B / dt, "tflops": flops / dt / 1e12,
                    "algorithmic_bytes_per_step": bytes_, "hbm_GBs_if_algorithmic": bytes_ / dt / 1e9,
                    "frac_of_hbm_peak": bytes_ / dt / 1e9 / PEAK_HBM_GBS})
        print(f"[bench] ae training {name}: {1e3 * dt:.3f} ms/step", file=sys.stderr, flush=True)
        del tr, X
    res = {"workload": "480x480, 4x4: one interior and one interface autoencoder of the largest subdomain, "
                       "width 2N, band 9, minibatch 64, BF16 MFMA + FP32 masters/Adam, synthetic snapshots",
           "steps_timed": 50, "autoencoders": out}
    res["fom_snapshot_training"] = cfg3_training(torch, dr)
    return res


def cfg3_training(torch, dr):
    """GPU training on the FOM snapshots of the 480x480, 4x4 workload (1024 snapshots on a 32 x 32
    parameter grid, 10% held out), for the largest subdomain's interior and interface
    autoencoders (models/cfg3_slice.npz, raw states in FP32): the recipe (2000 epochs at most,
    minibatch 64, plateau decay, early stopping), and a run of the same seed, split, initial
    weights and minibatch order for the epochs of the FP64 CPU-trained reference
    (models/cfg3_ae_ref_<part><k>.json), whose held-out reconstruction error it is set beside."""
    from paper_2305_15163_amd.train_ae import train_ae
    from paper_2305_15163_amd.train_model import decode_full, encode, unpack_weights
    import seeded_inputs as si
    files = [f for f in [os.path.join(ROOT, "models", "cfg3_slice.npz")] if os.path.exists(f)]
    if not files:
        print("[bench] no FOM snapshot slices of the 480x480 workload: GPU training on snapshots skipped",
              file=sys.stderr, flush=True)
        return None
    data = dict(np.load(files[0], allow_pickle=False))
    k = int(data["sd"])
    out = {"subdomain": k, "snapshots": int(data["X_om"].shape[0]), "data": "raw FOM states stored in FP32",
           "autoencoders": []}
    for part, n in (("om", 8), ("ga", 4)):
        X = np.asarray(data[f"X_{part}"], dtype=np.float64)
        seed = int(data[f"seed_{part}"])
        N = X.shape[1]
        runs = {}
        ref_path = os.path.join(ROOT, "models", f"cfg3_ae_ref_{part}{k}.json")
        ref = json.load(open(ref_path)) if os.path.exists(ref_path) else None
        # the recipe in BF16; the reference's epoch count in BF16 and in split-BF16 (FP32-class
        # products), each with the recipe's schedule (plateau decay, early stopping)
        plan = [("recipe", 2000, 0)] + ([("same_as_cpu_reference", int(ref["epochs"]), 0),
                                          ("same_as_cpu_reference_split_bf16", int(ref["epochs"]), 1)] if ref else [])
        for tag, epochs, prec in plan:
            t0 = time.perf_counter()
            r = train_ae(X, n, 9, 2, 0, seed, epochs, batch=64, precision=prec)
            dt = time.perf_counter() - t0
            w = unpack_weights(r.packed, N, n, 9, 2)
            g = si.rng(seed)
            perm = g.permutation(X.shape[0])
            n_test = max(1, int(round(0.1 * X.shape[0])))
            Xt = X[perm[:n_test]]
            rec = decode_full(w, encode(w, (Xt - r.mid) / r.scale, 2 * N, 0), N, 9, 2, 0) * r.scale + r.mid
            rel = np.linalg.norm(rec - Xt, axis=1) / np.linalg.norm(Xt, axis=1)
            steps = r.epochs * -(-(X.shape[0] - n_test) // 64)
            runs[tag] = {"epochs": r.epochs, "precision": ("bf16", "split_bf16")[prec], "seconds": dt,
                         "steps_per_s": steps / dt,
                         "best_test_loss": r.best_test, "rel_rec_err_mean": float(rel.mean()),
                         "rel_rec_err_max": float(rel.max())}
            print(f"[bench] cfg3 {part}{k} GPU {tag}: {r.epochs} epochs in {dt:.1f}s, held-out rel. error "
                  f"{rel.mean():.3e}", file=sys.stderr, flush=True)
        if ref:
            runs["cpu_fp64_reference"] = {key: ref[key] for key in ("epochs", "seconds", "best_test_loss",
                                                                     "rel_rec_err_mean", "rel_rec_err_max")}
        out["autoencoders"].append({"part": part, "N": N, "latent": n, "seed": seed, **runs})
    return out


PAPER = dict(pack="paper_gpu.npz", ref="paper", batch=512, seed=7, lam_range=(5.0, 25.0),
             # latent sizes, GPU-trained pack, the paper's error at mu* (Section 7.6 table)
             sweep=((4, 2, "paper_gpu_L4.npz", 7.04e-3), (6, 3, "paper_gpu_L6.npz", 2.60e-3),
                    (8, 4, "paper_gpu.npz", 1.64e-3), (10, 5, "paper_gpu_L10.npz", 1.19e-3),
                    (16, 8, "paper_gpu_L16.npz", 9.80e-4)),
             workload="the paper's own workload (Sections 7.1-7.3, 7.6): Burgers 480x24 on [-1,1]x[0,0.05], 2x2 "
                      "subdomains, latents (8,4), Swish, band-5 shift-5 masks, 100 HR nodes per subdomain, "
                      "autoencoders trained on the GPU (6400 snapshots, 80x80 grid, 2000 epochs at most)")


def paper_leg(a, torch, dr, si):
    """The paper's workload with GPU-trained autoencoders: the error against the FOM at the
    paper's test point mu* and over 64 held-out parameters, under the paper's stopping rule
    (||F|| < 1e-4 or 15 iterations, FP64) and under the batch rule of the headline (FP32
    decoders); batched throughput of 512 held-out parameters; plain B = 1 solves."""
    path = os.path.join(ROOT, "models", PAPER["pack"])
    if not os.path.exists(path):
        print(f"[bench] paper-scale leg skipped: missing {path}", file=sys.stderr, flush=True)
        return None
    pack = dict(np.load(path, allow_pickle=False))
    model = dr.Model(pack)
    B = PAPER["batch"]
    mu_h = si.heldout_mu(B, PAPER["seed"], lam_range=PAPER["lam_range"])
    star = np.array([[7692.5384, 21.9230]])
    X_star, X_held = fom_reference(PAPER["ref"], [("star", star), ("heldout", mu_h[:64])])
    rules = {"paper_f64": dr.opts(max_iter=15, tol_abs=1e-4, tol_rel=0.0, precision=0),
             "batch_rule_f32": dr.opts(max_iter=60, tol_rel=1e-6, precision=1, stall_tol=1e-5, stall_ratio=0.5)}
    out = {"workload": PAPER["workload"], "n_D": model.n_D, "n_C": model.n_C, "batch": B}
    ws, ws1 = dr.Workspace(model, B), dr.Workspace(model, 1)
    mu = torch.as_tensor(mu_h, device="cuda")
    for tag, o in rules.items():
        leg = {}
        dr.rom_solve_batch(model, ws, mu, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            r = dr.rom_solve_batch(model, ws, mu, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = {k: v.cpu().numpy() for k, v in r.items()}
        leg["batched"] = {"solves_per_s": B * a.steps / dt, "iters_mean": float(res["iters"].mean()),
                          "status_counts": {dr.STATUS[k]: int((res["status"] == k).sum())
                                            for k in np.unique(res["status"])}}
        rs = dr.rom_solve_batch(model, ws1, torch.as_tensor(star, device="cuda"), o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n1 = 16
        for b in range(n1):
            dr.rom_solve_batch(model, ws1, mu[b:b + 1], o)
        torch.cuda.synchronize()
        leg["plain_b1_solves_per_s"] = n1 / (time.perf_counter() - t0)
        leg["mu_star"] = {"status": dr.STATUS[int(rs["status"][0])], "iters": int(rs["iters"][0])}
        if X_star is not None:
            e = dr.relative_error(model, ws1, rs["xhat"], torch.as_tensor(X_star, device="cuda")).cpu().numpy()
            leg["mu_star"]["rel_err_vs_fom"] = float(e[0])
        if X_held is not None:
            w64 = dr.Workspace(model, 64)
            e = dr.relative_error(model, w64, torch.as_tensor(res["xhat"][:64], device="cuda"),
                                  torch.as_tensor(X_held, device="cuda")).cpu().numpy()
            leg["rel_err_vs_fom"] = error_summary(e, res["status"][:64], dr)
        out[tag] = leg
        print(f"[bench] paper-scale ({tag}): {leg['batched']['solves_per_s']:.0f} solves/s, mu* error "
              f"{leg['mu_star'].get('rel_err_vs_fom', float('nan')):.3e}", file=sys.stderr, flush=True)
    out["paper_reported_rel_err_mu_star"] = 1.64e-3
    # the latent sweep of the paper's Section 7.6 table, where its GPU-trained packs exist
    sweep = []
    for (n_om, n_ga, fname, paper_err) in PAPER["sweep"]:
        spath = os.path.join(ROOT, "models", fname)
        if not os.path.exists(spath):
            continue
        sm = dr.Model(dict(np.load(spath, allow_pickle=False)))
        sws1, sws64 = dr.Workspace(sm, 1), dr.Workspace(sm, 64)
        row = {"latents": [n_om, n_ga], "pack": fname, "paper_rel_err_mu_star": paper_err}
        rs = dr.rom_solve_batch(sm, sws1, torch.as_tensor(star, device="cuda"), rules["paper_f64"])
        if X_star is not None:
            row["rel_err_mu_star"] = float(dr.relative_error(sm, sws1, rs["xhat"],
                                                             torch.as_tensor(X_star, device="cuda")).cpu()[0])
        row["mu_star_status"] = dr.STATUS[int(rs["status"][0])]
        if X_held is not None:
            r64 = dr.rom_solve_batch(sm, sws64, mu[:64], rules["batch_rule_f32"])
            e = dr.relative_error(sm, sws64, r64["xhat"], torch.as_tensor(X_held, device="cuda")).cpu().numpy()
            row["rel_err_vs_fom_64"] = error_summary(e, r64["status"].cpu().numpy(), dr)
        sweep.append(row)
        print(f"[bench] paper-scale latents ({n_om},{n_ga}): mu* error {row.get('rel_err_mu_star', float('nan')):.3e} "
              f"(paper {paper_err:.2e})", file=sys.stderr, flush=True)
    out["latent_sweep"] = sweep
    # the same path without hyper-reduction (every owned node sampled)
    npath = os.path.join(ROOT, "models", "paper_gpu_nohr.npz")
    if os.path.exists(npath) and X_star is not None:
        nm_ = dr.Model(dict(np.load(npath, allow_pickle=False)))
        nws1 = dr.Workspace(nm_, 1)
        rs = dr.rom_solve_batch(nm_, nws1, torch.as_tensor(star, device="cuda"), rules["paper_f64"])
        out["without_hr"] = {"pack": "paper_gpu_nohr.npz", "paper_rel_err_mu_star": 1.28e-3,
                             "mu_star_status": dr.STATUS[int(rs["status"][0])],
                             "rel_err_mu_star": float(dr.relative_error(nm_, nws1, rs["xhat"], torch.as_tensor(
                                 X_star, device="cuda")).cpu()[0])}
        print(f"[bench] paper-scale without HR: mu* error {out['without_hr']['rel_err_mu_star']:.3e} (paper 1.28e-3)",
              file=sys.stderr, flush=True)
    # the LS-ROM contrast of Section 7.6 (POD maps of the same snapshots, latents (8,4), the same
    # HR nodes and C, collocation)
    lpath = os.path.join(ROOT, "models", "paper_ls.npz")
    if os.path.exists(lpath):
        lm = dr.Model(dict(np.load(lpath, allow_pickle=False)))
        lws1, lws = dr.Workspace(lm, 1), dr.Workspace(lm, B)
        ls = {"pack": "paper_ls.npz", "paper_rel_err_mu_star": 1.44e-2}
        rs = dr.rom_solve_batch(lm, lws1, torch.as_tensor(star, device="cuda"), rules["paper_f64"])
        ls["mu_star_status"] = dr.STATUS[int(rs["status"][0])]
        if X_star is not None:
            ls["rel_err_mu_star"] = float(dr.relative_error(lm, lws1, rs["xhat"],
                                                            torch.as_tensor(X_star, device="cuda")).cpu()[0])
        dr.rom_solve_batch(lm, lws, mu, rules["batch_rule_f32"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            rl = dr.rom_solve_batch(lm, lws, mu, rules["batch_rule_f32"])
        torch.cuda.synchronize()
        ls["batched_solves_per_s"] = B * a.steps / (time.perf_counter() - t0)
        if X_held is not None:
            w64 = dr.Workspace(lm, 64)
            e = dr.relative_error(lm, w64, rl["xhat"][:64].contiguous(), torch.as_tensor(X_held, device="cuda")).cpu().numpy()
            ls["rel_err_vs_fom_64"] = error_summary(e, rl["status"][:64].cpu().numpy(), dr)
        out["lsrom"] = ls
        print(f"[bench] paper-scale LS-ROM: mu* error {ls.get('rel_err_mu_star', float('nan')):.3e} (paper 1.44e-2), "
              f"{ls['batched_solves_per_s']:.0f} solves/s", file=sys.stderr, flush=True)
    return out


def roofline_only(a, torch, dr, si):
    """The dominant kernel's 20 all-live timing launches of the headline workload, then 5 device
    copies of 256 MiB (torch copy kernel: 256 MiB read and 256 MiB written each), whose byte
    counters calibrate FETCH_SIZE / WRITE_SIZE readings to bytes."""
    from paper_2305_15163_amd import autotune
    cfg = CONFIGS["cfg1"]
    pack = dict(np.load(os.path.join(ROOT, "models", "cfg1.npz"), allow_pickle=False))
    torch.cuda.set_device(0)
    B = cfg["batch"]
    mu_h = si.heldout_mu(B, cfg["seed"])
    o = dr.opts(max_iter=cfg["max_iter"], tol_rel=cfg["tol_rel"], precision=cfg["precision"],
                stall_tol=cfg["stall_tol"], stall_ratio=cfg["stall_ratio"])
    tile = autotune.tiles_for(pack, mu_h, o, path=os.path.join(ROOT, "paper_2305_15163_amd", "tiles.json"))
    model = dr.Model(pack, tile=tile)
    ws = dr.Workspace(model, B)
    mu = torch.as_tensor(mu_h, device="cuda")
    ms = dr.time_kernels(model, ws, mu, torch.zeros((B, model.n_D), dtype=torch.float64, device="cuda"),
                         precision=cfg["precision"], reps=20)
    n = 64 << 20
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    flops, bytes_ = decoder_work(model, B)
    print(json.dumps({"roofline_workload": "cfg1 interior decoder, 20 timing launches (B=512, all live)",
                      "work_item_shape": list(model.tile),
                      "ms_per_launch": ms, "algorithmic_bytes_per_launch": bytes_, "flops_per_launch": flops,
                      "copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n}), flush=True)


# Child program for the all-core oracle rate: one worker process per core, BLAS limited to one
# thread each, every worker solving its own share of the held-out parameters for about `secs`
# seconds after loading the model.  It never touches the GPU.
_CPU_ALL = r"""
import json, os, sys, time
for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[v] = "1"
sys.path.insert(0, sys.argv[1])
import numpy as np
from multiprocessing import Pool

def work(args):
    w, n, path, max_iter, secs, B, seed = args
    import seeded_inputs as si
    from oracle.pack import load_pack
    from oracle.rom import SQPOptions, sqp_solve
    om = load_pack(dict(np.load(path, allow_pickle=False)))
    mu = si.heldout_mu(B, seed)
    t0 = time.perf_counter(); k = 0
    while True:
        sqp_solve(om, mu[(w + k * n) % len(mu)], opts=SQPOptions(max_iter=max_iter, tol_abs=0.0, tol_rel=1e-8))
        k += 1
        if time.perf_counter() - t0 > secs:
            break
    return k, time.perf_counter() - t0

n, path, max_iter, secs = int(sys.argv[2]), sys.argv[3], int(sys.argv[4]), float(sys.argv[5])
B, seed = int(sys.argv[6]), int(sys.argv[7])
with Pool(n) as pool:
    res = pool.map(work, [(w, n, path, max_iter, secs, B, seed) for w in range(n)])
print(json.dumps({"solves": sum(k for k, _ in res), "rate": sum(k / t for k, t in res)}))
"""


def cpu_all_cores(path, max_iter, B, seed, secs=10.0):
    import subprocess
    n = min(os.cpu_count() or 1, 16)
    r = subprocess.run([sys.executable, "-c", _CPU_ALL, ROOT, str(n), path, str(max_iter), str(secs), str(B),
                        str(seed)],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("all-core oracle run failed: " + r.stderr[-2000:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": d["rate"], "unit": "solves/s", "cores": n, "solves": d["solves"], "cpu_model": model,
            "sample": f"{n} processes, one per core, BLAS limited to 1 thread each, about {secs:.0f} s each, "
                      f"held-out parameters of the 240x240 workload"}


def fom_reference(name, sets):
    """Stored FOM reference states (models/<name>_fomref.npz, written by the offline FOM
    reference script): for each (set name, parameters) pair, the states [n][N_x] if the file
    holds exactly those parameters, else None."""
    path = os.path.join(ROOT, "models", f"{name}_fomref.npz")
    if not os.path.exists(path):
        print(f"[bench] no FOM reference states at {path} (python -m oracle.fom_reference ...): error "
              f"against the FOM not measured", file=sys.stderr, flush=True)
        return [None] * len(sets)
    ref = np.load(path, allow_pickle=False)
    out = []
    for sname, mus in sets:
        key = f"{sname}_mu"
        if key in ref and ref[key].shape == np.shape(mus) and np.array_equal(ref[key], mus):
            out.append(np.asarray(ref[f"{sname}_x"], dtype=np.float64))
        else:
            print(f"[bench] {path}: set {sname} does not hold the benchmark's parameters", file=sys.stderr,
                  flush=True)
            out.append(None)
    return out


# Child program for the FOM's Newton time on one host core (the paper's speedup denominator), run
# inside the CPU-baseline leg: a few monolithic solves of held-out parameters.  It never touches
# the GPU.
_FOM_TIME = r"""
import os, sys, time, json
for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[v] = "1"
sys.path.insert(0, sys.argv[1])
import numpy as np
from oracle.burgers import BurgersFOM, Grid, solve_fom
nx, ny, k = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
mus = np.load(sys.argv[5])[:k]
fom = BurgersFOM(Grid(nx, ny))
t0 = time.perf_counter()
ok = all(solve_fom(fom, tuple(m)).converged for m in mus)
print(json.dumps({"s_per_solve": (time.perf_counter() - t0) / len(mus), "n": len(mus), "converged": ok}))
"""


def fom_newton_time(mus, nx, ny, k=3):
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "mu.npy")
        np.save(src, np.ascontiguousarray(mus, dtype=np.float64))
        r = subprocess.run([sys.executable, "-c", _FOM_TIME, ROOT, str(nx), str(ny), str(k), src],
                           capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError("FOM timing run failed: " + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def error_summary(err, status, dr):
    """eq. relative_error against the FOM over a subset of solves, overall and split by status."""
    err = np.asarray(err, dtype=np.float64)
    status = np.asarray(status)
    out = {"n": int(len(err)), "mean": float(err.mean()), "median": float(np.median(err)),
           "max": float(err.max()), "by_status": {}}
    for k in np.unique(status):
        e = err[status == k]
        out["by_status"][dr.STATUS[int(k)]] = {"n": int(len(e)), "mean": float(e.mean()), "max": float(e.max())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg1")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--plain", type=int, default=64, help="parameters for the plain per-solve GPU SQP legs")
    ap.add_argument("--n-err", type=int, default=64, help="parameters per leg for the error against the FOM")
    ap.add_argument("--proposal-batch", type=int, default=2048, help="held-out parameters of the proposal leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the three-model uneven batch leg")
    ap.add_argument("--uneven-only", action="store_true", help="run only the three-model uneven batch leg")
    ap.add_argument("--uneven-cpu-packs", action="store_true",
                    help="uneven leg on the CPU-trained packs even where GPU-trained ones exist")
    ap.add_argument("--no-ae", action="store_true", help="skip the autoencoder training leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-scale leg")
    ap.add_argument("--paper-only", action="store_true", help="run only the paper-scale leg")
    ap.add_argument("--ae-only", action="store_true", help="run only the autoencoder training leg")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the dominant kernel's timing launches and a device copy of known size "
                         "(the workload of the hardware-counter runs)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(parameter solves would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_15163_amd as dr
    import seeded_inputs as si

    if a.roofline_only:
        roofline_only(a, torch, dr, si)
        return

    if a.ae_only:
        torch.cuda.set_device(0)
        res = ae_training_leg(a, torch, dr, si)
        # five 256 MiB device copies: what FETCH_SIZE / WRITE_SIZE read for known bytes
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"ae_training": res}), flush=True)
        return

    if a.paper_only:
        torch.cuda.set_device(0)
        print(json.dumps({"paper_scale": paper_leg(a, torch, dr, si)}), flush=True)
        return

    if a.uneven_only:
        torch.cuda.set_device(0)
        print(json.dumps({"uneven_batch": uneven_leg(a, torch, dr)}), flush=True)
        return

    cfg = CONFIGS[a.config]
    path = os.path.join(ROOT, "models", f"{a.config}.npz")
    if not os.path.exists(path):
        print(f"missing model pack {path}; build it with: python -m oracle.build_model {a.config}", file=sys.stderr)
        sys.exit(1)
    pack = dict(np.load(path, allow_pickle=False))
    torch.cuda.set_device(0)
    print(f"[bench] loading model {path}", file=sys.stderr, flush=True)
    B = cfg["batch"]
    mu_h = si.heldout_mu(B, cfg["seed"])
    mu = torch.as_tensor(mu_h, device="cuda")
    o = dr.opts(max_iter=cfg["max_iter"], tol_rel=cfg["tol_rel"], precision=cfg["precision"],
                stall_tol=cfg["stall_tol"], stall_ratio=cfg["stall_ratio"])
    # work-item shapes from the persisted table of measured shapes (measured now when missing)
    from paper_2305_15163_amd import autotune
    tile = autotune.tiles_for(pack, mu_h, o, path=os.path.join(ROOT, "paper_2305_15163_amd", "tiles.json"),
                              verbose=True)
    model = dr.Model(pack, tile=tile)
    ws = dr.Workspace(model, B)
    f = dict(dtype=torch.float64, device="cuda")
    out = dict(xhat=torch.empty((B, model.n_D), **f), lam=torch.empty((B, max(1, model.n_C)), **f),
               iters=torch.empty((B,), dtype=torch.int32, device="cuda"),
               status=torch.empty((B,), dtype=torch.int32, device="cuda"),
               fnorm=torch.empty((B,), **f), fnorm0=torch.empty((B,), **f))

    out["fallback"] = torch.empty((B,), dtype=torch.int32, device="cuda")
    ppath = os.path.join(ROOT, "models", f"{a.config}_mlp.npz")
    prop = dr.Proposal.from_pack(dict(np.load(ppath, allow_pickle=False))) if os.path.exists(ppath) else None
    if prop is None:
        print(f"[bench] no proposal at {ppath}: zero start only", file=sys.stderr, flush=True)

    def run_cold():
        dr.rom_solve_batch(model, ws, mu, o, out=out)

    def run_warm():
        dr.rom_solve_warm(model, ws, prop, mu, o, out=out)

    def timed(fn, tag):
        for w in range(a.warmup):
            fn()
            torch.cuda.synchronize()
            print(f"[bench] {tag} warmup {w + 1}/{a.warmup} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(a.steps):
            fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench] {tag}: timed {a.steps} steps in {dt:.3f}s", file=sys.stderr, flush=True)
        res = {k: v.cpu().numpy().copy() for k, v in out.items()}
        return dt, res

    dt_c, res_c = timed(run_cold, "zero start")
    cold = {"solves_per_s": B * a.steps / dt_c, "ms_per_step": 1e3 * dt_c / a.steps,
            "iters_mean": float(res_c["iters"].mean()), "iters_max": int(res_c["iters"].max()),
            "status_counts": {dr.STATUS[k]: int((res_c["status"] == k).sum()) for k in np.unique(res_c["status"])}}
    if prop is not None:
        dt, res = timed(run_warm, "warm start")
    else:
        dt, res = dt_c, res_c
    value = B * a.steps / dt
    iters = res["iters"]
    status = res["status"]
    xb = res["xhat"]

    # dominant kernel: interior decoder subnets, every solve live
    ms = dr.time_kernels(model, ws, mu, torch.zeros((B, model.n_D), **f), precision=cfg["precision"], reps=20)
    flops, bytes_ = decoder_work(model, B)
    achieved = flops / (ms[0] * 1e-3) / 1e12
    if cfg["precision"] == 1:
        roof = {"bound": "alu", "kernel": "k_decode<float,8,...> (interior subnets, all solves live)",
                "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS}
    else:
        roof = {"bound": "alu", "kernel": "k_decode<double,...> (interior subnets, all solves live)",
                "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VECTOR_TFLOPS}
    dc = DECODE_COUNTERS
    if (cfg["precision"] == 1 and a.config == "cfg1" and decoder_source_sha1() == dc["source_sha1"]
            and tuple(model.tile) == dc["tile"]):
        roof["traffic"] = 1024.0 * (dc["fetch_kib"] * dc["fetch_scale"] + dc["write_kib"] * dc["write_scale"])
        roof["traffic_source"] = dc["profile"]
    else:
        roof["traffic"] = None
    roof["algorithmic_bytes_per_launch"] = bytes_
    roof["hbm_GBs_if_algorithmic"] = bytes_ / (ms[0] * 1e-3) / 1e9
    roof["ms_per_launch"] = {"decode_interior": ms[0], "decode_interface": ms[1], "residual_gn": ms[2], "constraint": ms[3]}
    print(f"[bench] kernel ms {ms}", file=sys.stderr, flush=True)

    # plain per-solve GPU SQP: B = 1, zero start, sequential host calls; once in FP64 at the
    # relative tolerance 1e-8, once at the batch's own precision and stopping rule
    plain, px, pst, px32, pst32 = None, None, None, None, None
    a.plain = min(a.plain, B)
    if a.plain > 0:
        ws1 = dr.Workspace(model, 1)
        legs = {}
        for tag, o1 in (("f64", dr.opts(max_iter=cfg["max_iter"], tol_rel=1e-8, precision=0)), ("batch_precision", o)):
            dr.rom_solve_batch(model, ws1, mu[:1], o1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            outs = [dr.rom_solve_batch(model, ws1, mu[b:b + 1], o1) for b in range(a.plain)]
            torch.cuda.synchronize()
            pt = time.perf_counter() - t1
            xs = torch.cat([r["xhat"] for r in outs]).cpu().numpy()
            ss = torch.cat([r["status"] for r in outs]).cpu().numpy()
            its = torch.cat([r["iters"] for r in outs]).cpu().numpy()
            legs[tag] = {"solves_per_s": a.plain / pt, "n": a.plain, "batch": 1, "iters_mean": float(its.mean()),
                         "status_counts": {dr.STATUS[k]: int((ss == k).sum()) for k in np.unique(ss)}}
            if tag == "f64":
                px, pst = xs, ss
                legs[tag].update(precision="f64", stop="||F|| <= 1e-8 ||F0||")
            else:
                px32, pst32 = xs, ss
                legs[tag].update(precision="f32+f64", stop=line_stop(cfg))
            print(f"[bench] plain per-solve SQP ({tag}) {legs[tag]['solves_per_s']:.1f} solves/s", file=sys.stderr,
                  flush=True)
        plain = legs["f64"]
        plain["same_precision_leg"] = legs["batch_precision"]

    # learned-proposal leg at its own workload size: 2048 held-out parameters, warm start vs zero start
    prop_leg = None
    if prop is not None and a.proposal_batch > 0:
        Bq = a.proposal_batch
        mu_q_h = si.heldout_mu(Bq, cfg["proposal_seed"])
        mu_q = torch.as_tensor(mu_q_h, device="cuda")
        wsq = dr.Workspace(model, Bq)
        res_q = {}
        for tag, fn in (("warm", lambda: dr.rom_solve_warm(model, wsq, prop, mu_q, o)),
                        ("zero_start", lambda: dr.rom_solve_batch(model, wsq, mu_q, o))):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(a.steps):
                r = fn()
            torch.cuda.synchronize()
            dtq = time.perf_counter() - t1
            rq = {k: v.cpu().numpy().copy() for k, v in r.items()}
            res_q[tag] = rq
            res_q[tag + "_rate"] = {"solves_per_s": Bq * a.steps / dtq, "iters_mean": float(rq["iters"].mean()),
                                    "iters_max": int(rq["iters"].max()),
                                    "status_counts": {dr.STATUS[k]: int((rq["status"] == k).sum())
                                                      for k in np.unique(rq["status"])}}
        prop_leg = {"workload": f"{Bq} held-out (a,lambda) (seed {cfg['proposal_seed']}), same model and options",
                    "warm": res_q["warm_rate"], "zero_start": res_q["zero_start_rate"],
                    "fallback_count": int(res_q["warm"]["fallback"].sum())}
        print(f"[bench] proposal leg: warm {prop_leg['warm']['solves_per_s']:.0f} solves/s, zero start "
              f"{prop_leg['zero_start']['solves_per_s']:.0f}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if cfg["precision"] == 1 else "f64", "data": "synthetic",
        "config": {"workload": cfg["workload"], "batch": B, "subdomains": model.n_sub, "n_D": model.n_D,
                   "work_item_shape": list(model.tile), "n_C": model.n_C, "stop": line_stop(cfg),
                   "start": ("learned proposal, zero-start fallback" if prop is not None else "zero start")},
        "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
        "status_counts": {dr.STATUS[k]: int((status == k).sum()) for k in np.unique(status)},
        "fallback_count": int(res["fallback"].sum()) if prop is not None else None,
        "zero_start": cold,
        "roofline": roof,
        "plain_sqp": plain,
        "speedup_vs_plain": (value / plain["solves_per_s"]) if plain else None,
        "speedup_vs_plain_same_precision": (value / plain["same_precision_leg"]["solves_per_s"]) if plain else None,
        "proposal": prop_leg,
    }

    if not a.no_uneven:
        line["uneven_batch"] = uneven_leg(a, torch, dr)
    if not a.no_ae:
        line["ae_training"] = ae_training_leg(a, torch, dr, si)
    if not a.no_paper:
        line["paper_scale"] = paper_leg(a, torch, dr, si)

    # error against the FOM (eq. relative_error) on the first n_err parameters of each leg, from
    # the stored FOM reference states of those parameters
    X_batch, X_prop = None, None
    if a.n_err > 0:
        n_err = min(a.n_err, B)
        sets = [("batch", mu_h[:n_err])]
        if prop_leg is not None:
            sets.append(("proposal", mu_q_h[:min(a.n_err, Bq)]))
        refs = fom_reference(a.config, sets)
        X_batch = refs[0]
        X_prop = refs[1] if prop_leg is not None else None
    if X_batch is not None:
        wse = dr.Workspace(model, n_err)
        Xf_d = torch.as_tensor(X_batch, device="cuda")

        def errs(xh):
            return dr.relative_error(model, wse, torch.as_tensor(xh[:n_err], device="cuda"), Xf_d).cpu().numpy()

        e_b, e_z = errs(xb), errs(res_c["xhat"])
        rel = {"n": n_err, "subset": f"the first {n_err} of the {B} held-out parameters",
               "batched": error_summary(e_b, status[:n_err], dr),
               "zero_start_batch": error_summary(e_z, res_c["status"][:n_err], dr)}
        if px is not None:
            m = min(n_err, len(px))
            e_p, e_p32 = errs(px)[:m], errs(px32)[:m]
            rel["plain_f64"] = error_summary(e_p, pst[:m], dr)
            rel["plain_same_precision"] = error_summary(e_p32, pst32[:m], dr)
            ratio = e_b[:m] / e_p
            rel["batched_over_plain_f64"] = {"max": float(ratio.max()), "median": float(np.median(ratio)),
                                             "within_1.1": int((ratio <= 1.1).sum()), "n": m}
        if prop_leg is not None and X_prop is not None:
            nq = min(a.n_err, Bq)
            Xq_d = torch.as_tensor(X_prop, device="cuda")
            wsq2 = dr.Workspace(model, nq)
            e_w = dr.relative_error(model, wsq2, torch.as_tensor(res_q["warm"]["xhat"][:nq], device="cuda"),
                                    Xq_d).cpu().numpy()
            e_q0 = dr.relative_error(model, wsq2, torch.as_tensor(res_q["zero_start"]["xhat"][:nq], device="cuda"),
                                     Xq_d).cpu().numpy()
            prop_leg["rel_err_vs_fom"] = {"n": nq, "warm": error_summary(e_w, res_q["warm"]["status"][:nq], dr),
                                          "zero_start": error_summary(e_q0, res_q["zero_start"]["status"][:nq], dr)}
        line["rel_err_vs_fom"] = rel
        line["rel_err_vs_fom"]["reference"] = f"models/{a.config}_fomref.npz (FP64 FOM Newton states, stored in FP32)"
        # LS-ROM contrast (Section 3.3): POD maps on the same grid, split, latents, HR nodes and
        # C, with collocation and with gappy-POD HR, same batch, options and FOM references
        ls = {}
        for tag, fname in (("collocation", f"{a.config}ls.npz"), ("gappy_pod", f"{a.config}lsg.npz")):
            lpath = os.path.join(ROOT, "models", fname)
            if not os.path.exists(lpath):
                continue
            lpack = dict(np.load(lpath, allow_pickle=False))
            lm = dr.Model(lpack)
            lws = dr.Workspace(lm, B)
            dr.rom_solve_batch(lm, lws, mu, o)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            for _ in range(a.steps):
                lr = dr.rom_solve_batch(lm, lws, mu, o)
            torch.cuda.synchronize()
            ldt = time.perf_counter() - t3
            lres = {k: v.cpu().numpy() for k, v in lr.items()}
            lwse = dr.Workspace(lm, n_err)
            le = dr.relative_error(lm, lwse, torch.as_tensor(lres["xhat"][:n_err], device="cuda"), Xf_d).cpu().numpy()
            ls[tag] = {"model": fname, "solves_per_s": B * a.steps / ldt, "iters_mean": float(lres["iters"].mean()),
                       "status_counts": {dr.STATUS[k]: int((lres["status"] == k).sum())
                                         for k in np.unique(lres["status"])},
                       "rel_err_vs_fom": error_summary(le, lres["status"][:n_err], dr)}
            print(f"[bench] LS-ROM ({tag}) {ls[tag]['solves_per_s']:.0f} solves/s", file=sys.stderr, flush=True)
        if ls:
            line["lsrom"] = dict(ls, workload="LS-ROM (POD maps, latents as the NM-ROM) on the same grid, split, "
                                              "HR nodes and C; same batch, precision and stopping rule")

    if not a.no_cpu:
        from threadpoolctl import threadpool_limits
        from oracle.pack import load_pack
        from oracle.rom import SQPOptions, sqp_solve
        om = load_pack(pack)
        with threadpool_limits(limits=1):
            t2 = time.perf_counter()
            n_cpu, ref = 0, []
            while True:
                ref.append(sqp_solve(om, mu_h[n_cpu], opts=SQPOptions(max_iter=cfg["max_iter"], tol_abs=0.0,
                                                                      tol_rel=1e-8)))
                n_cpu += 1
                if time.perf_counter() - t2 > 10.0 or n_cpu >= B:
                    break
            ct = time.perf_counter() - t2
        line["cpu_baseline"] = {"value": n_cpu / ct, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "sample": f"{n_cpu} of the {B} parameters, FP64 oracle SQP (dense KKT), "
                                          f"relative KKT tolerance 1e-8, BLAS limited to 1 thread"}
        if px is not None:
            # the oracle's solves of the same parameters against the plain FP64 GPU solves
            m = min(n_cpu, len(px))
            d = [float(np.max(np.abs(px[b] - ref[b].xhat)) / max(1e-300, np.max(np.abs(ref[b].xhat))))
                 for b in range(m)]
            line["oracle_vs_plain_f64"] = {"n": m, "max_rel_diff_xhat": max(d),
                                           "status_equal": int(sum(int(pst[b]) == ref[b].status for b in range(m)))}
            print(f"[bench] oracle vs plain FP64 GPU solves: max rel diff {max(d):.2e} over {m}", file=sys.stderr,
                  flush=True)
        print(f"[bench] cpu leg {n_cpu} solves in {ct:.1f}s", file=sys.stderr, flush=True)
        # the FOM's Newton solve per parameter on one host core (the paper's speedup denominator)
        ft = fom_newton_time(mu_h, *model_grid(pack), k=3)
        line["cpu_baseline"]["fom_newton"] = {"s_per_solve": ft["s_per_solve"], "n": ft["n"], "cores": 1,
                                              "batched_solves_per_fom_solve_time": line["value"] * ft["s_per_solve"]}
        print(f"[bench] FOM Newton {ft['s_per_solve']:.2f} s per solve on one core", file=sys.stderr, flush=True)
        line["cpu_baseline"]["all_cores"] = cpu_all_cores(path, cfg["max_iter"], B, cfg["seed"])
        print(f"[bench] all-core oracle leg: {line['cpu_baseline']['all_cores']['value']:.2f} solves/s on "
              f"{line['cpu_baseline']['all_cores']['cores']} cores", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


def line_stop(cfg):
    out = (f"||F|| <= {cfg['tol_rel']:g} ||F0||, max_iter {cfg['max_iter']}, "
           f"or stagnation below {cfg['stall_tol']:g} ||F0|| (Armijo failure")
    if cfg.get("stall_ratio", 0.0) > 0.0:
        out += f", or an accepted step reducing ||F|| by less than the factor {cfg['stall_ratio']:g}"
    return out + ")"


def model_grid(pack):
    return int(pack["nx"]), int(pack["ny"])


if __name__ == "__main__":
    main()
