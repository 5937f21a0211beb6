"""ctypes binding of libddrom.so (argument marshalling only; every step of the solve runs
in the library's HIP kernels).  PyTorch supplies device memory and the stream.

The library is built in-tree (see build.py); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddrom.so")

PREC_FP64 = 0
PREC_FP32_DECODER = 1

STATUS = {0: "converged", 1: "max_iter", 2: "linesearch_fail", 3: "kkt_not_pd", 4: "nonfinite", 5: "stalled"}


class DecoderDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("n", C.c_int), ("w", C.c_int), ("b", C.c_int), ("s", C.c_int),
                ("W1", C.POINTER(C.c_double)), ("b1", C.POINTER(C.c_double)),
                ("W2", C.POINTER(C.c_double)), ("x_ref", C.POINTER(C.c_double)), ("dense", C.c_int)]


class ModelDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nu", C.c_double), ("ly", C.c_double),
                ("nsx", C.c_int), ("nsy", C.c_int), ("activation", C.c_int), ("n_C", C.c_int), ("N_A", C.c_int),
                ("C", C.POINTER(C.c_double)), ("dec_om", C.POINTER(DecoderDesc)), ("dec_ga", C.POINTER(DecoderDesc)),
                ("hr_count", C.POINTER(C.c_int)), ("hr_nodes", C.POINTER(C.POINTER(C.c_int))),
                ("tile", C.c_int * 3), ("n_ports", C.c_int), ("dec_port", C.POINTER(DecoderDesc)),
                ("port_activation", C.c_int), ("hr_modes", C.POINTER(C.c_int)),
                ("hr_gappy", C.POINTER(C.POINTER(C.c_double)))]


class MlpDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("sizes", C.POINTER(C.c_int)), ("params", C.POINTER(C.c_float)),
                ("out_mean", C.POINTER(C.c_double)), ("out_std", C.POINTER(C.c_double)), ("n_D", C.c_int)]


class Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol_abs", C.c_double), ("tol_rel", C.c_double), ("armijo_c1", C.c_double),
                ("max_backtracks", C.c_int), ("precision", C.c_int), ("stall_tol", C.c_double),
                ("stall_ratio", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2305_15163_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
        L.ddrom_last_error.restype = C.c_char_p
        L.ddrom_model_create.argtypes = [C.POINTER(ModelDesc), C.POINTER(vp)]
        L.ddrom_model_destroy.argtypes = [vp]
        L.ddrom_model_size.argtypes = [vp, ip, ip]
        L.ddrom_model_size.restype = C.c_longlong
        L.ddrom_subnet_rows.argtypes = [vp, ip, ip, C.POINTER(C.c_int)]
        L.ddrom_workspace_create.argtypes = [vp, ip, C.POINTER(vp)]
        L.ddrom_workspace_destroy.argtypes = [vp]
        L.dd_fom_residual.argtypes = [vp, vp, vp, ip, vp, vp, vp]
        L.ae_decode_hr.argtypes = [vp, vp, ip, ip, vp, ip, ip, vp, vp]
        L.ae_jacobian_hr.argtypes = [vp, vp, ip, ip, vp, ip, ip, vp, vp, vp]
        L.ae_jacobian_hr_noalloc.argtypes = [vp, ip, ip, vp, ip, ip, vp, vp, vp]
        L.ddrom_gn_blocks.argtypes = [vp, vp, vp, vp, ip, ip, vp, vp, vp, vp, vp, vp]
        L.sqp_step.argtypes = [vp, vp, vp, ip, vp, vp, vp, vp, C.POINTER(Opts), vp]
        L.rom_solve_batch.argtypes = [vp, vp, vp, ip, vp, vp, C.POINTER(Opts), vp, vp, vp, vp, vp, vp, vp]
        L.ddrom_time_kernels.argtypes = [vp, vp, vp, vp, ip, ip, ip, C.POINTER(C.c_float)]
        L.ddrom_mlp_create.argtypes = [C.POINTER(MlpDesc), C.POINTER(vp)]
        L.ddrom_mlp_destroy.argtypes = [vp]
        L.ddrom_mlp_size.argtypes = [vp, ip]
        L.ddrom_mlp_size.restype = C.c_longlong
        L.mlp_proposal.argtypes = [vp, vp, ip, vp, vp, vp]
        L.ddrom_mlp_trainer_create.argtypes = [C.POINTER(MlpDesc), ip, C.POINTER(vp)]
        L.ddrom_mlp_trainer_destroy.argtypes = [vp]
        L.ddrom_mlp_trainer_size.argtypes = [vp, ip]
        L.ddrom_mlp_trainer_size.restype = C.c_longlong
        L.ddrom_mlp_trainer_params.argtypes = [vp, vp, vp]
        L.mlp_train_step.argtypes = [vp, vp, vp, vp, ip, C.c_float, ip, vp, vp, vp]
        L.rom_solve_warm.argtypes = [vp, vp, vp, vp, ip, C.POINTER(Opts), vp, vp, vp, vp, vp, vp, vp, vp]
        L.rom_decode_states.argtypes = [vp, vp, vp, ip, ip, vp, vp]
        L.ddrom_autotune.argtypes = [C.POINTER(ModelDesc), vp, ip, C.POINTER(Opts), ip, C.POINTER(C.c_int),
                                     C.POINTER(C.c_float), ip, C.POINTER(C.c_int)]
        L.rom_solve_multi.argtypes = [ip, vp, vp, vp, vp, C.POINTER(Opts), vp, vp, vp, vp, vp, vp]
        L.ddrom_ae_trainer_create.argtypes = [ip, ip, ip, ip, ip, ip, ip, C.POINTER(C.c_float), C.POINTER(vp)]
        L.ddrom_ae_trainer_destroy.argtypes = [vp]
        L.ddrom_ae_trainer_size.argtypes = [vp, ip]
        L.ddrom_ae_trainer_size.restype = C.c_longlong
        L.ddrom_ae_trainer_params.argtypes = [vp, vp, vp]
        L.ae_train_step.argtypes = [vp, vp, vp, ip, vp, C.c_float, ip, vp, vp, vp]
        L.rom_relative_error.argtypes = [vp, vp, vp, ip, ip, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed ({rc}): {lib().ddrom_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    """Device tensors handed to the library by pointer must be contiguous CUDA tensors of the
    stated dtype (a strided view would be read with the wrong layout)."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    return t


def _dev(x, dtype=torch.float64):
    t = torch.as_tensor(x, dtype=dtype)
    return t.to("cuda").contiguous()


def model_desc(pack: dict, tile=(0, 0, 0)):
    """ddrom_model_desc of a model pack; the second value holds the host arrays it points to."""
    n = int(pack["n_sub"])
    keep = []

    def dptr(a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def desc(prefix):
        if f"{prefix}_Phi" in pack:
            # LS-ROM affine map x0 + Phi xhat as a dense decoder: W1 = I, b1 = 0, identity activation
            Phi = np.asarray(pack[f"{prefix}_Phi"], dtype=np.float64)
            N, n = Phi.shape
            return DecoderDesc(N, n, n, 0, 0, dptr(np.eye(n)), dptr(np.zeros(n)), dptr(Phi),
                               dptr(pack[f"{prefix}_x0"]), 1)
        W1 = np.asarray(pack[f"{prefix}_W1"])
        b, s = (int(v) for v in pack[f"{prefix}_bs"])
        N = int(np.asarray(pack[f"{prefix}_xref"]).shape[0])
        return DecoderDesc(N, int(W1.shape[1]) if W1.ndim == 2 else 0, int(W1.shape[0]), b, s, dptr(W1),
                           dptr(pack[f"{prefix}_b1"]), dptr(pack[f"{prefix}_W2"]), dptr(pack[f"{prefix}_xref"]), 0)

    srpc = int(pack.get("srpc", 0)) == 1
    n_ports = int(pack["n_ports"]) if srpc else 0
    decs = {}
    for part in (("om",) if srpc else ("om", "ga")):
        arr = (DecoderDesc * n)()
        for i in range(n):
            arr[i] = desc(f"{part}{i}")
        decs[part] = arr
    ports = (DecoderDesc * max(1, n_ports))()
    for j in range(n_ports):
        ports[j] = desc(f"pt{j}")
    keep.extend([decs, ports])
    hr = [np.ascontiguousarray(np.asarray(pack[f"hr{i}"], dtype=np.int32)) for i in range(n)]
    keep.extend(hr)
    hr_cnt = (C.c_int * n)(*[len(h) for h in hr])
    hr_ptrs = (C.POINTER(C.c_int) * n)(*[h.ctypes.data_as(C.POINTER(C.c_int)) for h in hr])
    keep.extend([hr_cnt, hr_ptrs])
    Cm = np.asarray(pack["C"], dtype=np.float64)
    # gappy-POD hyper-reduction: gp{i}_P = (Z_i Phi_i^r)^+ [n_r][2 N_B]
    if "gp0_P" in pack:
        gp = [np.asarray(pack[f"gp{i}_P"], dtype=np.float64) for i in range(n)]
        g_modes = (C.c_int * n)(*[int(P.shape[0]) for P in gp])
        g_ptrs = (C.POINTER(C.c_double) * n)(*[dptr(P) for P in gp])
        keep.extend([g_modes, g_ptrs])
    else:
        g_modes, g_ptrs = C.POINTER(C.c_int)(), C.POINTER(C.POINTER(C.c_double))()
    desc = ModelDesc(int(pack["nx"]), int(pack["ny"]), float(pack["nu"]), float(pack["ly"]), int(pack["nsx"]),
                     int(pack["nsy"]), int(pack["act"]), int(Cm.shape[0]), int(Cm.shape[1]), dptr(Cm),
                     decs["om"], decs["ga"] if not srpc else C.POINTER(DecoderDesc)(), hr_cnt, hr_ptrs,
                     (C.c_int * 3)(*[int(v) for v in tile]), n_ports, ports,
                     int(pack["port_act"]) if srpc else 0, g_modes, g_ptrs)
    return desc, keep


class Model:
    """Device model built from a model pack (dict of numpy arrays, see oracle.pack's format).
    tile = (decoder rows, residual nodes, constraint rows) per work item, 0 for the default."""

    def __init__(self, pack: dict, tile=(0, 0, 0)):
        L = lib()
        n = int(pack["n_sub"])
        desc, keep = model_desc(pack, tile)
        h = C.c_void_p()
        _check(L.ddrom_model_create(C.byref(desc), C.byref(h)), "ddrom_model_create")
        self.h = h
        self.n_sub = n
        self.n_D = self.size(1)
        self.n_C = self.size(2)
        self.N_A = self.size(3)
        self.N_x = self.size(4)
        self.n_state = self.size(5)
        self.n_om = [self.size(10, i) for i in range(n)]
        self.n_ga = [self.size(11, i) for i in range(n)]
        self.N_om = [self.size(12, i) for i in range(n)]
        self.N_ga = [self.size(13, i) for i in range(n)]
        self.xoff = [self.size(17, i) for i in range(n)]
        self.tile = (self.size(7), self.size(8), self.size(9))

    def size(self, q, sd=-1):
        return int(lib().ddrom_model_size(self.h, q, sd))

    def subnet_rows(self, sd, part=0):
        n = self.size(14, sd) if part == 0 else self.N_ga[sd]
        out = (C.c_int * max(1, n))()
        _check(lib().ddrom_subnet_rows(self.h, sd, part, out), "ddrom_subnet_rows")
        return np.array(out[:n], dtype=np.int64)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ddrom_model_destroy(self.h)
            self.h = None


class Workspace:
    def __init__(self, model: Model, max_batch: int):
        self.model = model
        self.max_batch = max_batch
        h = C.c_void_p()
        _check(lib().ddrom_workspace_create(model.h, int(max_batch), C.byref(h)), "ddrom_workspace_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ddrom_workspace_destroy(self.h)
            self.h = None


def opts(max_iter=50, tol_abs=0.0, tol_rel=1e-8, armijo_c1=1e-4, max_backtracks=20, precision=PREC_FP64,
         stall_tol=0.0, stall_ratio=0.0) -> Opts:
    return Opts(int(max_iter), float(tol_abs), float(tol_rel), float(armijo_c1), int(max_backtracks), int(precision),
                float(stall_tol), float(stall_ratio))


def dd_fom_residual(model: Model, mu, xsd, jac: bool = False):
    mu, xsd = _dev(mu), _dev(xsd)
    B = mu.shape[0]
    r = torch.empty((B, model.N_x), dtype=torch.float64, device="cuda")
    J = torch.empty((B, model.N_x, 6), dtype=torch.float64, device="cuda") if jac else None
    _check(lib().dd_fom_residual(model.h, _ptr(mu), _ptr(xsd), B, _ptr(r), _ptr(J), _stream()), "dd_fom_residual")
    return (r, J) if jac else r


def ae_jacobian_hr(model: Model, ws: Workspace, sd: int, part: int, xhat, precision=PREC_FP64, want_x=True):
    xhat = _dev(xhat)
    B = xhat.shape[0]
    rows = model.size(14, sd) if part == 0 else model.N_ga[sd]
    n = model.n_om[sd] if part == 0 else model.n_ga[sd]
    dt = torch.float64 if precision == PREC_FP64 else torch.float32
    x = torch.empty((B, rows), dtype=dt, device="cuda") if want_x else None
    J = torch.empty((B, rows, n), dtype=dt, device="cuda")
    _check(lib().ae_jacobian_hr(model.h, ws.h, sd, part, _ptr(xhat), B, precision, _ptr(x), _ptr(J), _stream()),
           "ae_jacobian_hr")
    return x, J


def ae_jacobian_hr_noalloc(model: Model, sd: int, part: int, xhat, x, J, precision=PREC_FP64):
    """ae_jacobian_hr without a workspace, into caller-allocated x [B][rows] (or None) and
    J [B][rows][n] of the precision's dtype; the library allocates nothing."""
    xhat = _need(xhat, torch.float64, "xhat")
    dt = torch.float64 if precision == PREC_FP64 else torch.float32
    if x is not None:
        _need(x, dt, "x")
    _need(J, dt, "J")
    _check(lib().ae_jacobian_hr_noalloc(model.h, sd, part, _ptr(xhat), xhat.shape[0], precision, _ptr(x), _ptr(J),
                                        _stream()), "ae_jacobian_hr_noalloc")
    return x, J


def ae_decode_hr(model: Model, ws: Workspace, sd: int, part: int, xhat, precision=PREC_FP64):
    xhat = _dev(xhat)
    B = xhat.shape[0]
    rows = model.size(14, sd) if part == 0 else model.N_ga[sd]
    dt = torch.float64 if precision == PREC_FP64 else torch.float32
    x = torch.empty((B, rows), dtype=dt, device="cuda")
    _check(lib().ae_decode_hr(model.h, ws.h, sd, part, _ptr(xhat), B, precision, _ptr(x), _stream()), "ae_decode_hr")
    return x


def gn_blocks(model: Model, ws: Workspace, mu, xhat, precision=PREC_FP64):
    mu, xhat = _dev(mu), _dev(xhat)
    B = mu.shape[0]
    nmax = max(a + b for a, b in zip(model.n_om, model.n_ga))
    mmax = max(1, max(model.n_ga))
    f = dict(dtype=torch.float64, device="cuda")
    H = torch.zeros((B, model.n_sub, nmax, nmax), **f)
    g = torch.zeros((B, model.n_D), **f)
    EG = torch.zeros((B, model.n_sub, model.n_C, mmax), **f)
    c = torch.zeros((B, max(1, model.n_C)), **f)
    rr = torch.zeros((B,), **f)
    _check(lib().ddrom_gn_blocks(model.h, ws.h, _ptr(mu), _ptr(xhat), B, precision, _ptr(H), _ptr(g), _ptr(EG),
                                 _ptr(c), _ptr(rr), _stream()), "ddrom_gn_blocks")
    return H, g, EG, c[:, :model.n_C], rr


def sqp_step(model: Model, ws: Workspace, mu, xhat, lam, o: Opts):
    mu = _dev(mu)
    x = _dev(xhat).clone()
    l = _dev(lam).clone()
    B = mu.shape[0]
    fn = torch.empty((B,), dtype=torch.float64, device="cuda")
    st = torch.empty((B,), dtype=torch.int32, device="cuda")
    _check(lib().sqp_step(model.h, ws.h, _ptr(mu), B, _ptr(x), _ptr(l), _ptr(fn), _ptr(st), C.byref(o), _stream()),
           "sqp_step")
    return x, l, fn, st


def rom_solve_batch(model: Model, ws: Workspace, mu, o: Opts, xhat0=None, lam0=None, out=None):
    """Returns dict(xhat, lam, iters, status, fnorm, fnorm0) of device tensors.  `out` may
    pass preallocated tensors with those keys (the call then allocates nothing)."""
    mu = _dev(mu)
    B = mu.shape[0]
    x0 = None if xhat0 is None else _dev(xhat0)
    l0 = None if lam0 is None else _dev(lam0)
    if out is None:
        f = dict(dtype=torch.float64, device="cuda")
        out = dict(xhat=torch.empty((B, model.n_D), **f), lam=torch.empty((B, max(1, model.n_C)), **f),
                   iters=torch.empty((B,), dtype=torch.int32, device="cuda"),
                   status=torch.empty((B,), dtype=torch.int32, device="cuda"),
                   fnorm=torch.empty((B,), **f), fnorm0=torch.empty((B,), **f))
    _check(lib().rom_solve_batch(model.h, ws.h, _ptr(mu), B, _ptr(x0), _ptr(l0), C.byref(o), _ptr(out["xhat"]),
                                 _ptr(out["lam"]), _ptr(out["iters"]), _ptr(out["status"]), _ptr(out["fnorm"]),
                                 _ptr(out["fnorm0"]), _stream()), "rom_solve_batch")
    return out


def time_kernels(model: Model, ws: Workspace, mu, xhat, precision=PREC_FP32_DECODER, reps=20):
    """Average ms per launch of [interior decode, interface decode, residual+GN, constraint]."""
    mu, xhat = _dev(mu), _dev(xhat)
    B = mu.shape[0]
    ms = (C.c_float * 4)()
    _check(lib().ddrom_time_kernels(model.h, ws.h, _ptr(mu), _ptr(xhat), B, precision, reps, ms), "ddrom_time_kernels")
    return list(ms)


# ---- learned initial iterate ---------------------------------------------------------

def pack_mlp_params(layers) -> np.ndarray:
    """[(W [out][in], b [out]), ...] -> the packed FP32 parameter vector of ddrom_mlp_desc."""
    return np.concatenate([np.concatenate([np.asarray(W, dtype=np.float32).ravel(), np.asarray(b, dtype=np.float32)])
                           for W, b in layers])


def unpack_mlp_params(flat, sizes) -> list:
    flat = np.asarray(flat)
    out, o = [], 0
    for k in range(len(sizes) - 1):
        fi, fo = sizes[k], sizes[k + 1]
        W = flat[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = flat[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def _mlp_desc(sizes, params, out_mean, out_std, n_D, keep):
    sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    pr = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    n_out = int(sz[-1])
    mn = np.ascontiguousarray(np.zeros(n_out) if out_mean is None else np.asarray(out_mean, dtype=np.float64))
    sd = np.ascontiguousarray(np.ones(n_out) if out_std is None else np.asarray(out_std, dtype=np.float64))
    keep += [sz, pr, mn, sd]
    return MlpDesc(len(sz) - 1, sz.ctypes.data_as(C.POINTER(C.c_int)), pr.ctypes.data_as(C.POINTER(C.c_float)),
                   mn.ctypes.data_as(C.POINTER(C.c_double)), sd.ctypes.data_as(C.POINTER(C.c_double)), int(n_D))


class Proposal:
    """Device copy of a trained proposal network (see mlp_proposal in include/ddrom.h)."""

    def __init__(self, sizes, params, out_mean, out_std, n_D: int):
        keep = []
        d = _mlp_desc(sizes, params, out_mean, out_std, n_D, keep)
        h = C.c_void_p()
        _check(lib().ddrom_mlp_create(C.byref(d), C.byref(h)), "ddrom_mlp_create")
        self.h = h
        self.sizes = [int(v) for v in sizes]
        self.n_D = int(n_D)
        self.n_out = self.sizes[-1]

    @classmethod
    def from_pack(cls, pk: dict):
        return cls(pk["sizes"], pk["params"], pk["out_mean"], pk["out_std"], int(pk["n_D"]))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ddrom_mlp_destroy(self.h)
            self.h = None


class ProposalTrainer:
    """FP32 trainer of the proposal network (forward, back-propagation and Adam in HIP)."""

    def __init__(self, sizes, params, max_batch: int):
        keep = []
        d = _mlp_desc(sizes, params, None, None, 0, keep)
        h = C.c_void_p()
        _check(lib().ddrom_mlp_trainer_create(C.byref(d), int(max_batch), C.byref(h)), "ddrom_mlp_trainer_create")
        self.h = h
        self.sizes = [int(v) for v in sizes]
        self.n_params = int(lib().ddrom_mlp_trainer_size(h, 0))
        self.max_batch = int(max_batch)

    def step(self, mu, target, rows, lr: float = 1e-3, update: bool = True, loss: bool = False, grad: bool = False):
        """One minibatch; mu [N][2] FP64, target [N][out] FP32 (standardised), rows [B] int32,
        all contiguous device tensors.  Returns (loss tensor or None, gradient tensor or None)."""
        _need(mu, torch.float64, "mu")
        _need(target, torch.float32, "target")
        _need(rows, torch.int32, "rows")
        B = int(rows.shape[0])
        lt = torch.empty((1,), dtype=torch.float32, device="cuda") if loss else None
        gt = torch.empty((self.n_params,), dtype=torch.float32, device="cuda") if grad else None
        _check(lib().mlp_train_step(self.h, _ptr(mu), _ptr(target), _ptr(rows), B, float(lr), int(bool(update)),
                                    _ptr(lt), _ptr(gt), _stream()), "mlp_train_step")
        return lt, gt

    def params(self):
        out = torch.empty((self.n_params,), dtype=torch.float32, device="cuda")
        _check(lib().ddrom_mlp_trainer_params(self.h, _ptr(out), _stream()), "ddrom_mlp_trainer_params")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ddrom_mlp_trainer_destroy(self.h)
            self.h = None


def mlp_proposal(p: Proposal, mu):
    """(xhat0 [B][n_D], lam0 [B][outputs - n_D]) proposed for parameters mu [B][2]."""
    mu = _dev(mu)
    B = mu.shape[0]
    f = dict(dtype=torch.float64, device="cuda")
    x0 = torch.empty((B, p.n_D), **f)
    l0 = torch.empty((B, max(1, p.n_out - p.n_D)), **f)
    _check(lib().mlp_proposal(p.h, _ptr(mu), B, _ptr(x0), _ptr(l0), _stream()), "mlp_proposal")
    return x0, l0[:, :p.n_out - p.n_D]


def rom_solve_warm(model: Model, ws: Workspace, p: Proposal, mu, o: Opts, out=None):
    """rom_solve_batch warm-started from the proposal (zero start as fallback).  Returns
    dict(xhat, lam, iters, status, fnorm, fnorm0, fallback) of device tensors."""
    mu = _dev(mu)
    B = mu.shape[0]
    if out is None:
        f = dict(dtype=torch.float64, device="cuda")
        i32 = dict(dtype=torch.int32, device="cuda")
        out = dict(xhat=torch.empty((B, model.n_D), **f), lam=torch.empty((B, max(1, model.n_C)), **f),
                   iters=torch.empty((B,), **i32), status=torch.empty((B,), **i32),
                   fnorm=torch.empty((B,), **f), fnorm0=torch.empty((B,), **f), fallback=torch.empty((B,), **i32))
    _check(lib().rom_solve_warm(model.h, ws.h, p.h, _ptr(mu), B, C.byref(o), _ptr(out["xhat"]), _ptr(out["lam"]),
                                _ptr(out["iters"]), _ptr(out["status"]), _ptr(out["fnorm"]), _ptr(out["fnorm0"]),
                                _ptr(out["fallback"]), _stream()), "rom_solve_warm")
    return out


# ---- after a solve -------------------------------------------------------------------

def decode_states(model: Model, ws: Workspace, xhat, precision=PREC_FP64):
    """Decoded DD states [B][n_state] (FP64) of latents xhat [B][n_D]."""
    xhat = _dev(xhat)
    B = xhat.shape[0]
    x = torch.empty((B, model.n_state), dtype=torch.float64, device="cuda")
    _check(lib().rom_decode_states(model.h, ws.h, _ptr(xhat), B, int(precision), _ptr(x), _stream()),
           "rom_decode_states")
    return x


def relative_error(model: Model, ws: Workspace, xhat, xfom, precision=PREC_FP64):
    """eq. relative_error of the decoded states of xhat [B][n_D] against FOM states xfom [B][N_x]."""
    xhat, xfom = _dev(xhat), _dev(xfom)
    B = xhat.shape[0]
    err = torch.empty((B,), dtype=torch.float64, device="cuda")
    _check(lib().rom_relative_error(model.h, ws.h, _ptr(xhat), B, int(precision), _ptr(xfom), _ptr(err), _stream()),
           "rom_relative_error")
    return err


# ---- autoencoder training ------------------------------------------------------------

def band_slots(N: int, b: int, s: int):
    """Column of every band slot [N][3][b] and its validity (inside [0, N s))."""
    r = np.arange(N)[:, None, None]
    k = np.arange(-1, 2)[None, :, None]
    t = np.arange(b)[None, None, :]
    cols = r * s + k * b * s + t
    return cols, (cols >= 0) & (cols < N * s)


def ae_pack(N: int, n: int, b: int, s: int, W1e_csr, b1e, W2e, W1d, b1d, W2d_csr) -> np.ndarray:
    """Packed trainer parameters from weights whose masked layers list their entries in row
    order of the mask (decoder: rows r, columns ascending) and of its transpose (encoder:
    hidden units c, inputs ascending)."""
    cols, valid = band_slots(N, b, s)
    flat_valid = np.flatnonzero(valid.ravel())
    w2d = np.zeros(3 * N * b)
    w2d[flat_valid] = np.asarray(W2d_csr)                       # row-major order == slot order
    rows = np.broadcast_to(np.arange(N)[:, None, None], cols.shape).ravel()[flat_valid]
    order = np.lexsort((rows, cols.ravel()[flat_valid]))        # encoder entries sorted by (c, r)
    w1e = np.zeros(3 * N * b)
    w1e[flat_valid[order]] = np.asarray(W1e_csr)
    return np.concatenate([w1e, b1e, np.asarray(W2e).ravel(), np.asarray(W1d).ravel(), b1d, w2d]).astype(np.float32)


def ae_unpack(flat, N: int, n: int, b: int, s: int):
    """Inverse of ae_pack: (W1e_csr, b1e, W2e, W1d, b1d, W2d_csr)."""
    flat = np.asarray(flat, dtype=np.float64)
    w = N * s
    nb = 3 * N * b
    o = [0, nb, nb + w, nb + w + n * w, nb + w + 2 * n * w, nb + 2 * w + 2 * n * w, 2 * nb + 2 * w + 2 * n * w]
    cols, valid = band_slots(N, b, s)
    flat_valid = np.flatnonzero(valid.ravel())
    rows = np.broadcast_to(np.arange(N)[:, None, None], cols.shape).ravel()[flat_valid]
    order = np.lexsort((rows, cols.ravel()[flat_valid]))
    w1e = flat[o[0]:o[1]][flat_valid[order]]
    w2d = flat[o[5]:o[6]][flat_valid]
    return (w1e, flat[o[1]:o[2]], flat[o[2]:o[3]].reshape(n, w), flat[o[3]:o[4]].reshape(w, n),
            flat[o[4]:o[5]], w2d)


class AETrainer:
    """GPU trainer of one band-masked autoencoder (BF16 matrix cores, FP32 masters, Adam)."""

    def __init__(self, N: int, n: int, b: int, s: int, activation: int, max_batch: int, packed, precision: int = 0):
        pr = np.ascontiguousarray(np.asarray(packed, dtype=np.float32))
        h = C.c_void_p()
        _check(lib().ddrom_ae_trainer_create(int(N), int(n), int(b), int(s), int(activation), int(max_batch),
                                             int(precision), pr.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)),
               "ddrom_ae_trainer_create")
        self.h = h
        self.N, self.n, self.b, self.s = int(N), int(n), int(b), int(s)
        self.n_params = int(lib().ddrom_ae_trainer_size(h, 0))

    def step(self, X, rows, scale, lr: float = 1e-3, update: bool = True, loss: bool = False, grad: bool = False):
        """X [n_snap][N], rows [B] (int32), scale [N]: contiguous FP32 device tensors."""
        _need(X, torch.float32, "X")
        _need(rows, torch.int32, "rows")
        _need(scale, torch.float32, "scale")
        if X.shape[-1] != self.N or scale.shape[0] != self.N:
            raise ValueError("snapshot width or scale length differs from the trainer's N")
        B = int(rows.shape[0])
        lt = torch.empty((1,), dtype=torch.float32, device="cuda") if loss else None
        gt = torch.empty((self.n_params,), dtype=torch.float32, device="cuda") if grad else None
        _check(lib().ae_train_step(self.h, _ptr(X), _ptr(rows), B, _ptr(scale), float(lr), int(bool(update)),
                                   _ptr(lt), _ptr(gt), _stream()), "ae_train_step")
        return lt, gt

    def params(self):
        out = torch.empty((self.n_params,), dtype=torch.float32, device="cuda")
        _check(lib().ddrom_ae_trainer_params(self.h, _ptr(out), _stream()), "ddrom_ae_trainer_params")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ddrom_ae_trainer_destroy(self.h)
            self.h = None


def rom_solve_multi(models, wss, mus, o: Opts):
    """Uneven batch over several models in one graph.  Returns one dict(xhat, lam, iters,
    status, fnorm) of device tensors per model."""
    k = len(models)
    mus = [_dev(m) for m in mus]
    f = dict(dtype=torch.float64, device="cuda")
    i32 = dict(dtype=torch.int32, device="cuda")
    outs = [dict(xhat=torch.empty((m_.shape[0], md.n_D), **f), lam=torch.empty((m_.shape[0], max(1, md.n_C)), **f),
                 iters=torch.empty((m_.shape[0],), **i32), status=torch.empty((m_.shape[0],), **i32),
                 fnorm=torch.empty((m_.shape[0],), **f)) for md, m_ in zip(models, mus)]
    vpa = C.c_void_p * k
    arr = lambda key: vpa(*[C.c_void_p(o_[key].data_ptr()) for o_ in outs])
    Bs = (C.c_int * k)(*[int(m_.shape[0]) for m_ in mus])
    _check(lib().rom_solve_multi(k, vpa(*[md.h for md in models]), vpa(*[w.h for w in wss]),
                                 vpa(*[C.c_void_p(m_.data_ptr()) for m_ in mus]), Bs, C.byref(o), arr("xhat"),
                                 arr("lam"), arr("iters"), arr("status"), arr("fnorm"), _stream()), "rom_solve_multi")
    return outs


def autotune_tiles(pack: dict, mu, o: Opts, reps: int = 5):
    """Work-item shape search (ddrom_autotune) for a model pack and a batch of parameters.
    Returns (tile, rows) with rows = [(dec rows, res nodes, con rows, ms), ...] as tried."""
    mu = _dev(mu)
    desc, keep = model_desc(pack)
    tile = (C.c_int * 3)()
    table = (C.c_float * (4 * 64))()
    n = C.c_int()
    _check(lib().ddrom_autotune(C.byref(desc), _ptr(mu), int(mu.shape[0]), C.byref(o), int(reps), tile, table, 64,
                                C.byref(n)), "ddrom_autotune")
    rows = [(int(table[4 * k]), int(table[4 * k + 1]), int(table[4 * k + 2]), float(table[4 * k + 3]))
            for k in range(min(64, n.value))]
    return tuple(int(v) for v in tile), rows
