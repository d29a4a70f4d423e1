"""ctypes binding of libpeps_hip.so (argument marshalling only) and the autograd wrapper.

Every computation runs in the HIP library; torch provides device memory and the
stream.  There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpeps_hip.so")

PREC = {"f64": 0, "f32": 1, "bf16": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP error",
          4: "unsupported", 5: "numerical failure"}


class PepsError(RuntimeError):
    pass


class _Lattice(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("D", ctypes.c_int32),
                ("Dc", ctypes.c_int32), ("J1", ctypes.c_double), ("J2", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("lat", _Lattice), ("A", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("batch", ctypes.c_int64), ("grad_mode", ctypes.c_int32),
                ("weights", ctypes.c_void_p), ("log_abs", ctypes.c_void_p),
                ("sign", ctypes.c_void_p), ("e_loc", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("flags", ctypes.c_void_p)]


_lib = None
_lock = threading.Lock()
_ctx = {}

_P = ctypes.c_void_p
_SIGS = {
    "peps_create": [ctypes.POINTER(_P), ctypes.c_int],
    "peps_destroy": [_P],
    "peps_set_stream": [_P, _P],
    "peps_set_workspace_limit": [_P, ctypes.c_size_t],
    "peps_set_fused_steps": [_P, ctypes.c_int32],
    "peps_set_truncation": [_P, ctypes.c_int32],
    "peps_workspace_query": [_P, ctypes.POINTER(_Lattice), ctypes.c_int64, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_size_t)],
    "peps_log_amplitude": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                           _P, _P, _P],
    "peps_local_energy": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                          _P, _P, _P, _P],
    "peps_log_derivative": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                            _P, _P, _P, _P, _P],
    "peps_plan_check": [ctypes.POINTER(_Lattice), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                        ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "peps_profile_enable": [_P, ctypes.c_uint32],
    "peps_profile_read": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "peps_profile_read_bytes": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "peps_eval_jobs": [_P, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_uint32],
    "peps_autotune": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                      ctypes.POINTER(ctypes.c_int32)],
    "peps_tune_save": [_P, ctypes.c_char_p],
    "peps_tune_load": [_P, ctypes.c_char_p],
    "peps_evaluate": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                      ctypes.c_int32, _P, _P, _P, _P, _P, _P],
    "peps_evaluate_noalloc": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                              ctypes.c_int32, _P, _P, _P, _P, _P, _P],
    "peps_metropolis_step": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                             _P, _P, _P, _P],
    "peps_go_update": [_P, ctypes.POINTER(_Lattice), _P, _P, _P, ctypes.c_double],
    "peps_pair_correlations": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64,
                               ctypes.c_int32, _P, _P, _P, _P],
    "peps_structure_factor": [_P, ctypes.POINTER(_Lattice), ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P],
    "peps_vmc_step": [_P, ctypes.POINTER(_Lattice), ctypes.c_int, _P, _P, ctypes.c_int64, ctypes.c_int32,
                      _P, _P, ctypes.c_double, _P, _P],
}


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise PepsError(f"{path} not found: build it with python -m paper_1806_03761_amd.build")
            lib = ctypes.CDLL(path)
            for name, args in _SIGS.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            lib.peps_last_error.argtypes = [_P]
            lib.peps_last_error.restype = ctypes.c_char_p
            lib.peps_noalloc_scratch_bytes.argtypes = []
            lib.peps_noalloc_scratch_bytes.restype = ctypes.c_size_t
            _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS) + ["peps_last_error", "peps_noalloc_scratch_bytes"]


def _context(device: int):
    lib = load_library()
    with _lock:
        c = _ctx.get(device)
        if c is None:
            h = _P()
            st = lib.peps_create(ctypes.byref(h), device)
            if st != 0:
                raise PepsError(f"peps_create({device}) failed: {STATUS.get(st, st)}")
            c = _ctx[device] = h
    return lib, c


def _check(lib, ctx, st, what):
    if st != 0:
        msg = lib.peps_last_error(ctx)
        raise PepsError(f"{what}: {STATUS.get(st, st)}: {msg.decode() if msg else ''}")


def _lat(lat) -> _Lattice:
    return _Lattice(int(lat.Lx), int(lat.Ly), int(lat.D), int(lat.Dc), float(lat.J1), float(lat.J2))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _prep(A, S, lat):
    if not (A.is_cuda and S.is_cuda):
        raise PepsError("A and S must be device tensors")
    if A.dtype != torch.float64 or S.dtype != torch.int8:
        raise PepsError("A must be float64 and S int8")
    N, D = lat.Lx * lat.Ly, lat.D
    if tuple(A.shape) != (N, 2, D, D, D, D):
        raise PepsError(f"A has shape {tuple(A.shape)}, expected {(N, 2, D, D, D, D)}")
    if S.dim() != 2 or S.shape[1] != N:
        raise PepsError(f"S has shape {tuple(S.shape)}, expected (batch, {N})")
    A = A.contiguous()
    S = S.contiguous()
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    lib, ctx = _context(dev)
    stream = torch.cuda.current_stream(A.device).cuda_stream
    lib.peps_set_stream(ctx, ctypes.c_void_p(stream))
    return lib, ctx, A, S


def plan_check(lat, batch: int, grad_mode: int = 3, want_eloc: bool = True, sweeps: int = 0) -> int:
    """Host-only dry run of the launch sequence with bounds checks (no GPU needed).
    Returns the workspace bytes of one chunk; raises if a bounds check fails."""
    lib = load_library()
    out = ctypes.c_size_t()
    st = lib.peps_plan_check(ctypes.byref(_lat(lat)), int(batch), int(grad_mode), int(bool(want_eloc)),
                             int(sweeps), ctypes.byref(out))
    if st != 0:
        raise PepsError(f"peps_plan_check failed: {STATUS.get(st, st)}")
    return int(out.value)


KERNEL_CLASS = {"gemm": 0, "qr": 1, "svd": 2, "fused": 3}


def profile_enable(classes=(), device: int = 0):
    """Time every launch of the given kernel classes ("gemm", "qr", "svd", "fused") with HIP
    events on the context's stream; () turns timing off."""
    lib, ctx = _context(device)
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASS[c]
    lib.peps_profile_enable(ctx, mask)


def profile_read(cls: str, device: int = 0):
    """(total device ms, launches, algorithmic flops) of one kernel class since enable."""
    lib, ctx = _context(device)
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    st = lib.peps_profile_read(ctx, KERNEL_CLASS[cls], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl))
    _check(lib, ctx, st, "peps_profile_read")
    return ms.value, n.value, fl.value


def profile_bytes(cls: str, device: int = 0) -> float:
    """Algorithmic HBM bytes of one kernel class's timed launches since enable (GEMM class;
    call after profile_read)."""
    lib, ctx = _context(device)
    by = ctypes.c_double()
    _check(lib, ctx, lib.peps_profile_read_bytes(ctx, KERNEL_CLASS[cls], ctypes.byref(by)),
           "peps_profile_read_bytes")
    return by.value


def autotune(A, S, lat, prec: str = "f32") -> int:
    """Pick the GEMM tile of every shape of this workload by timing (see peps_autotune)."""
    lib, ctx, A, S = _prep(A, S, lat)
    n = ctypes.c_int32()
    st = lib.peps_autotune(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), S.shape[0],
                           ctypes.byref(n))
    _check(lib, ctx, st, "peps_autotune")
    return int(n.value)


def tune_save(path: str, device: int = 0):
    lib, ctx = _context(device)
    _check(lib, ctx, lib.peps_tune_save(ctx, path.encode()), "peps_tune_save")


def tune_load(path: str, device: int = 0):
    lib, ctx = _context(device)
    _check(lib, ctx, lib.peps_tune_load(ctx, path.encode()), "peps_tune_load")


def set_truncation(sweeps: int, device: int = 0):
    """Boundary truncation of this device's context: 0 = canonical SVD (default),
    1..16 = variational compression with that many sweeps (see peps_set_truncation)."""
    lib, ctx = _context(device)
    _check(lib, ctx, lib.peps_set_truncation(ctx, int(sweeps)), "peps_set_truncation")


def set_fused_steps(enable: bool, device: int = 0):
    """Fused float32 sandwich steps on (default) or the GEMM form (same results)."""
    lib, ctx = _context(device)
    _check(lib, ctx, lib.peps_set_fused_steps(ctx, 1 if enable else 0), "peps_set_fused_steps")


def noalloc_scratch_bytes() -> int:
    """Size of the fixed device scratch array of peps_evaluate_noalloc."""
    return int(load_library().peps_noalloc_scratch_bytes())


def set_workspace_limit(nbytes: int, device: int = 0):
    lib, ctx = _context(device)
    lib.peps_set_workspace_limit(ctx, int(nbytes))


def workspace_bytes(lat, batch: int, prec: str = "f64", device: int = 0) -> int:
    lib, ctx = _context(device)
    out = ctypes.c_size_t()
    st = lib.peps_workspace_query(ctx, ctypes.byref(_lat(lat)), int(batch), PREC[prec], ctypes.byref(out))
    _check(lib, ctx, st, "peps_workspace_query")
    return int(out.value)


def log_amplitude(A, S, lat, prec: str = "f64"):
    """(log_abs float64 [B], sign int8 [B], flags int8 [B]) on A's device."""
    lib, ctx, A, S = _prep(A, S, lat)
    B = S.shape[0]
    la = torch.empty(B, dtype=torch.float64, device=A.device)
    sg = torch.empty(B, dtype=torch.int8, device=A.device)
    fl = torch.empty(B, dtype=torch.int8, device=A.device)
    st = lib.peps_log_amplitude(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B,
                                _ptr(la), _ptr(sg), _ptr(fl))
    _check(lib, ctx, st, "peps_log_amplitude")
    return la, sg, fl


def local_energy(A, S, lat, prec: str = "f64"):
    """(log_abs, sign, e_loc float64 [B], flags)."""
    lib, ctx, A, S = _prep(A, S, lat)
    B = S.shape[0]
    la = torch.empty(B, dtype=torch.float64, device=A.device)
    sg = torch.empty(B, dtype=torch.int8, device=A.device)
    e = torch.empty(B, dtype=torch.float64, device=A.device)
    fl = torch.empty(B, dtype=torch.int8, device=A.device)
    st = lib.peps_local_energy(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B,
                               _ptr(la), _ptr(sg), _ptr(e), _ptr(fl))
    _check(lib, ctx, st, "peps_local_energy")
    return la, sg, e, fl


def log_derivative(A, S, lat, prec: str = "f64", weights=None):
    """Per-sample Delta [B][N][2][D^4] (weights None) or sum_b weights[b] Delta_b [N][2][D^4]."""
    lib, ctx, A, S = _prep(A, S, lat)
    B = S.shape[0]
    N, D4 = lat.Lx * lat.Ly, lat.D ** 4
    if weights is not None:
        weights = weights.to(device=A.device, dtype=torch.float64).contiguous()
        if weights.shape != (B,):
            raise PepsError("weights must have shape (batch,)")
        out = torch.empty((N, 2, D4), dtype=torch.float64, device=A.device)
    else:
        out = torch.empty((B, N, 2, D4), dtype=torch.float64, device=A.device)
    la = torch.empty(B, dtype=torch.float64, device=A.device)
    sg = torch.empty(B, dtype=torch.int8, device=A.device)
    fl = torch.empty(B, dtype=torch.int8, device=A.device)
    st = lib.peps_log_derivative(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B,
                                 _ptr(weights), _ptr(out), _ptr(la), _ptr(sg), _ptr(fl))
    _check(lib, ctx, st, "peps_log_derivative")
    return out, la, sg, fl


def evaluate(A, S, lat, prec: str = "f64", grad_mode: int = 3, weights=None, out=None, noalloc=False):
    """Whole path from one set of environments: (log_abs, sign, e_loc, grad, flags).
    grad_mode 0 none, 1 per-sample, 2 weighted sum, 3 dE/dA of the energy estimator.
    noalloc: through peps_evaluate_noalloc (workspace in the library's fixed device
    scratch array instead of an allocated one)."""
    lib, ctx, A, S = _prep(A, S, lat)
    B = S.shape[0]
    N, D4 = lat.Lx * lat.Ly, lat.D ** 4
    dev = A.device
    la = torch.empty(B, dtype=torch.float64, device=dev)
    sg = torch.empty(B, dtype=torch.int8, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    fl = torch.empty(B, dtype=torch.int8, device=dev)
    if grad_mode and out is None:
        shape = (B, N, 2, D4) if grad_mode == 1 else (N, 2, D4)
        out = torch.empty(shape, dtype=torch.float64, device=dev)
    if weights is not None:
        weights = weights.to(device=dev, dtype=torch.float64).contiguous()
    fn = lib.peps_evaluate_noalloc if noalloc else lib.peps_evaluate
    st = fn(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B, grad_mode,
            _ptr(weights), _ptr(la), _ptr(sg), _ptr(e), _ptr(out), _ptr(fl))
    _check(lib, ctx, st, "peps_evaluate_noalloc" if noalloc else "peps_evaluate")
    return la, sg, e, out, fl


def metropolis_step(A, S, lat, u, log_abs, sign, prec: str = "f64", accepted=None):
    """One Metropolis step of every chain (peps_metropolis_step): S, log_abs and sign are
    updated in place; u is float64 [batch][2] of uniforms on the device.  Returns the int8
    accepted flags."""
    lib, ctx, A, S2 = _prep(A, S, lat)
    if S2.data_ptr() != S.data_ptr():
        raise PepsError("S must be contiguous: it is updated in place")
    B = S.shape[0]
    for t, dt, shape in ((u, torch.float64, (B, 2)), (log_abs, torch.float64, (B,)), (sign, torch.int8, (B,))):
        if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous() or t.device != S.device:
            raise PepsError(f"expected a contiguous {dt} tensor of shape {shape} on {S.device}")
    if accepted is None:
        accepted = torch.empty(B, dtype=torch.int8, device=A.device)
    st = lib.peps_metropolis_step(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B, _ptr(u),
                                  _ptr(log_abs), _ptr(sign), _ptr(accepted))
    _check(lib, ctx, st, "peps_metropolis_step")
    return accepted


def _param_like(t, A, what):
    if t.dtype != torch.float64 or t.numel() != A.numel() or not t.is_contiguous() or t.device != A.device:
        raise PepsError(f"{what} must be a contiguous float64 tensor with the elements of A, on {A.device}")


def go_update(A, grad, p, lat, dt: float):
    """GO update in place (peps_go_update): A -= p * dt * sign(grad), elementwise."""
    lib, ctx = _context(A.device.index or 0)
    for t, what in ((A, "A"), (grad, "grad"), (p, "p")):
        _param_like(t, A, what)
    N, D = lat.Lx * lat.Ly, lat.D
    if tuple(A.shape) != (N, 2, D, D, D, D):
        raise PepsError(f"A has shape {tuple(A.shape)}, expected {(N, 2, D, D, D, D)}")
    st = lib.peps_go_update(ctx, ctypes.byref(_lat(lat)), _ptr(A), _ptr(grad), _ptr(p), float(dt))
    _check(lib, ctx, st, "peps_go_update")
    return A


def vmc_step(A, S, lat, u, p, dt: float, prec: str = "f64", grad=None, return_grad: bool = True):
    """One optimisation-loop iteration in place (peps_vmc_step): u is float64
    [n_mc][batch][2] (n_mc may be 0), p shaped like A.  Returns (energy, grad) with
    energy a float64 device tensor {E, count} and grad dE/dA before the update (None
    with return_grad False: the library then keeps the gradient to itself)."""
    lib, ctx, A2, S2 = _prep(A, S, lat)
    if A2.data_ptr() != A.data_ptr() or S2.data_ptr() != S.data_ptr():
        raise PepsError("A and S must be contiguous: they are updated in place")
    B = S.shape[0]
    if u.dtype != torch.float64 or u.dim() != 3 or tuple(u.shape[1:]) != (B, 2) or not u.is_contiguous() \
            or u.device != A.device:
        raise PepsError(f"u must be a contiguous float64 tensor of shape (n_mc, {B}, 2)")
    _param_like(p, A, "p")
    if grad is None and return_grad:
        grad = torch.empty_like(A)
    if grad is not None:
        _param_like(grad, A, "grad")
    energy = torch.empty(2, dtype=torch.float64, device=A.device)
    st = lib.peps_vmc_step(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B, u.shape[0],
                           _ptr(u) if u.numel() else None, _ptr(p), float(dt), _ptr(energy), _ptr(grad))
    _check(lib, ctx, st, "peps_vmc_step")
    return energy, grad


def pair_correlations(A, S, lat, pairs, prec: str = "f64", per_sample: bool = False):
    """<S_m . S_n> for every (m, n) of `pairs` (peps_pair_correlations).  Returns
    (means [P], per-sample values [B][P] or None, flags [B]) as device tensors."""
    lib, ctx, A, S = _prep(A, S, lat)
    dev = A.device
    pr = torch.as_tensor(pairs, dtype=torch.int32).reshape(-1, 2).contiguous().to(dev)
    B, P = S.shape[0], pr.shape[0]
    means = torch.empty(P, dtype=torch.float64, device=dev)
    vals = torch.empty((B, P), dtype=torch.float64, device=dev) if per_sample else None
    fl = torch.empty(B, dtype=torch.int8, device=dev)
    st = lib.peps_pair_correlations(ctx, ctypes.byref(_lat(lat)), PREC[prec], _ptr(A), _ptr(S), B, P, _ptr(pr),
                                    _ptr(means), _ptr(vals), _ptr(fl))
    _check(lib, ctx, st, "peps_pair_correlations")
    return means, vals, fl


def structure_factor(corr, lat, sites, ks):
    """m_s^2(k) for each k of `ks` over `sites` from their correlation matrix
    (peps_structure_factor); corr is a float64 device tensor [n][n]."""
    lib, ctx = _context(corr.device.index or 0)
    sd = torch.as_tensor(sites, dtype=torch.int32).contiguous().to(corr.device)
    kd = torch.as_tensor(ks, dtype=torch.float64).reshape(-1, 2).contiguous().to(corr.device)
    n = sd.numel()
    if corr.dtype != torch.float64 or tuple(corr.shape) != (n, n) or not corr.is_contiguous():
        raise PepsError(f"corr must be a contiguous float64 tensor of shape {(n, n)}")
    out = torch.empty(kd.shape[0], dtype=torch.float64, device=corr.device)
    st = lib.peps_structure_factor(ctx, ctypes.byref(_lat(lat)), n, _ptr(sd), _ptr(corr), kd.shape[0], _ptr(kd),
                                   _ptr(out))
    _check(lib, ctx, st, "peps_structure_factor")
    return out


def correlation_matrix(A, S, lat, sites, prec: str = "f64"):
    """<S_i . S_j> over `sites`: pair_correlations on the unordered pairs i <= j, placed
    symmetrically into an [n][n] device tensor."""
    n = len(sites)
    iu = [(a, b) for a in range(n) for b in range(a, n)]
    means, _, fl = pair_correlations(A, S, lat, [(sites[a], sites[b]) for a, b in iu], prec)
    ia = torch.tensor([a for a, _ in iu], device=means.device)
    ib = torch.tensor([b for _, b in iu], device=means.device)
    C = torch.empty((n, n), dtype=torch.float64, device=means.device)
    C[ia, ib] = means
    C[ib, ia] = means
    return C, fl


def job_outputs(A, S, lat, grad_mode=3, want_eloc=True):
    """Preallocated outputs of one job: (log_abs, sign, e_loc or None, out or None, flags)."""
    B = S.shape[0]
    N, D4 = lat.Lx * lat.Ly, lat.D ** 4
    dev = A.device
    la = torch.empty(B, dtype=torch.float64, device=dev)
    sg = torch.empty(B, dtype=torch.int8, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev) if (want_eloc or grad_mode == 3) else None
    out = None
    if grad_mode:
        out = torch.empty((B, N, 2, D4) if grad_mode == 1 else (N, 2, D4), dtype=torch.float64, device=dev)
    fl = torch.empty(B, dtype=torch.int8, device=dev)
    return la, sg, e, out, fl


def eval_jobs(jobs, prec: str = "f32", graph: bool = True, outputs=None):
    """Several lattices in one call.  jobs: list of dicts with keys A, S, lat and optional
    grad_mode (default 3), weights, want_eloc (default True).  With graph=True the whole
    launch sequence is one HIP graph launch (replayed when the same tensors come again;
    pass the previous return value as `outputs` to reuse the output buffers).
    Returns one (log_abs, sign, e_loc, grad, flags) tuple per job."""
    if not jobs:
        return []
    arr = (_Job * len(jobs))()
    keep = []
    res = []
    lib = ctx = None
    for i, j in enumerate(jobs):
        lib, ctx, A, S = _prep(j["A"], j["S"], j["lat"])
        gm = int(j.get("grad_mode", 3))
        w = j.get("weights")
        if w is not None:
            w = w.to(device=A.device, dtype=torch.float64).contiguous()
        o = outputs[i] if outputs is not None else job_outputs(A, S, j["lat"], gm, j.get("want_eloc", True))
        la, sg, e, out, fl = o
        keep += [A, S, w]
        arr[i] = _Job(_lat(j["lat"]), _ptr(A), _ptr(S), S.shape[0], gm, _ptr(w), _ptr(la), _ptr(sg),
                      _ptr(e), _ptr(out), _ptr(fl))
        res.append(o)
    st = lib.peps_eval_jobs(ctx, ctypes.cast(arr, ctypes.c_void_p), len(jobs), PREC[prec], 1 if graph else 0)
    _check(lib, ctx, st, "peps_eval_jobs")
    eval_jobs._keep = keep          # inputs must outlive the enqueued work
    return res


class PepsLogAmp(torch.autograd.Function):
    """ln|W(S)| as a differentiable function of A; backward calls peps_log_derivative
    with the incoming gradient as per-sample weights (frozen environments)."""

    @staticmethod
    def forward(ctx, A, S, lat, prec="f64"):
        la, sg, fl = log_amplitude(A, S, lat, prec)
        ctx.save_for_backward(A, S)
        ctx.lat = lat
        ctx.prec = prec
        ctx.mark_non_differentiable(sg, fl)
        return la, sg, fl

    @staticmethod
    def backward(ctx, g, _gs=None, _gf=None):
        A, S = ctx.saved_tensors
        lat = ctx.lat
        gA = None
        if ctx.needs_input_grad[0]:
            out, _, _, _ = log_derivative(A, S, lat, ctx.prec, weights=g)
            gA = out.reshape(A.shape)
        return gA, None, None, None
