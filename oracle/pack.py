"""Model pack (.npz) -> oracle ROMModel.  The pack format is plain arrays:
grid (nx, ny, nu, ly), split (nsx, nsy), activation, n_sub, C, and per subdomain i and
part p in {om, ga}: p{i}_W1 [w, n], p{i}_b1 [w], p{i}_W2 [N, 3, b] band values,
p{i}_xref [N], p{i}_bs = (b, s); hr{i} = sampled global node ids (ascending).  A strong
ROM-port constraint pack (srpc = 1) has no interface decoders ga{i}; it holds one decoder per
port, pt{j}_* (ports in the DD maps' order, activation port_act), and an empty C."""
from __future__ import annotations

import numpy as np

from .autoencoder import Decoder
from .burgers import Grid
from .ddmaps import build_dd
from .rom import ROMModel
from .srpc import build_port_maps, interface_decoders


def load_pack(pack, use_hr: bool = True) -> ROMModel:
    if isinstance(pack, str):
        pack = dict(np.load(pack, allow_pickle=False))
    g = Grid(int(pack["nx"]), int(pack["ny"]), float(pack["nu"]), float(pack["ly"]))
    n = int(pack["n_sub"])
    act = int(pack["act"])
    dec = {}
    parts = ("om",) if int(pack.get("srpc", 0)) == 1 else ("om", "ga")
    for part in parts:
        dec[part] = []
        for i in range(n):
            b, s = (int(v) for v in pack[f"{part}{i}_bs"])
            dec[part].append(Decoder(np.asarray(pack[f"{part}{i}_W1"], np.float64), np.asarray(pack[f"{part}{i}_b1"], np.float64),
                                     np.asarray(pack[f"{part}{i}_W2"], np.float64), np.asarray(pack[f"{part}{i}_xref"], np.float64),
                                     b, s, act))
    hr = [np.asarray(pack[f"hr{i}"], np.int64) for i in range(n)] if use_hr else None
    if int(pack.get("srpc", 0)) == 1:
        return _srpc_model(pack, g, dec["om"], hr)
    return ROMModel(g, int(pack["nsx"]), int(pack["nsy"]), dec["om"], dec["ga"], hr, np.asarray(pack["C"], np.float64))


def _srpc_model(pack, g, dec_om, hr) -> ROMModel:
    """Strong ROM-port constraint pack: port decoders pt{j}_* (ports in the DD maps' order)
    instead of interface decoders; interface decoders and the constraint are implied."""
    dd = build_dd(g, int(pack["nsx"]), int(pack["nsy"]))
    n_ports = int(pack["n_ports"])
    if n_ports != len(dd.ports):
        raise ValueError("port count of the pack does not match the split")
    pact = int(pack["port_act"])
    pdec = []
    for j in range(n_ports):
        b, s = (int(v) for v in pack[f"pt{j}_bs"])
        pdec.append(Decoder(np.asarray(pack[f"pt{j}_W1"], np.float64), np.asarray(pack[f"pt{j}_b1"], np.float64),
                            np.asarray(pack[f"pt{j}_W2"], np.float64), np.asarray(pack[f"pt{j}_xref"], np.float64),
                            b, s, pact))
    pm = build_port_maps(dd, [d.n for d in pdec])
    dec_ga = interface_decoders(dd, pm, pdec)
    return ROMModel(g, int(pack["nsx"]), int(pack["nsy"]), dec_om, dec_ga, hr, np.zeros((0, dd.n_A)), dd=dd,
                    A_hat=pm.A_hat)


def load_ls_pack(pack, use_hr: bool = True):
    """LS-ROM pack (om{i}_Phi / om{i}_x0, ga{i}_Phi / ga{i}_x0 instead of decoders) -> the LS-ROM
    oracle with HR on the pack's nodes: collocation, or gappy POD when the pack carries the
    matrices gp{i}_P = (Z_i Phi_i^r)^+ (columns: r_u rows of the nodes, then r_v rows)."""
    from .burgers import BurgersFOM
    from .lsrom import LSROM, HROperator, collocation_operator
    if isinstance(pack, str):
        pack = dict(np.load(pack, allow_pickle=False))
    g = Grid(int(pack["nx"]), int(pack["ny"]), float(pack["nu"]), float(pack["ly"]))
    n = int(pack["n_sub"])
    dd = build_dd(g, int(pack["nsx"]), int(pack["nsy"]))
    get = lambda key: [np.asarray(pack[f"{key[0]}{i}_{key[1]}"], np.float64) for i in range(n)]
    hr = [collocation_operator(g, np.asarray(pack[f"hr{i}"], np.int64)) for i in range(n)] if use_hr else None
    if use_hr and "gp0_P" in pack:
        hr = [HROperator(op.rows, np.asarray(pack[f"gp{i}_P"], np.float64)) for i, op in enumerate(hr)]
    return LSROM(BurgersFOM(g), dd, np.asarray(pack["C"], np.float64), get(("om", "x0")), get(("om", "Phi")),
                 get(("ga", "x0")), get(("ga", "Phi")), hr=hr)
