"""Exact Hawkes log-likelihood and gradient on AMD Instinct MI355X (gfx950).

Thin Python binding of the C ABI in include/hawkes.h (libhawkes.so, built
from csrc/ by build.py).  It only marshals arguments: PyTorch provides the
device memory (tensors, workspace) and the stream; every step of the
computation runs in the library's HIP kernels.  If the library is missing
the functions raise; there is no CPU fallback.

Paper: "Massively Parallel Exact Inference for Hawkes Processes"
(arXiv 2604.01342), intensity eq. 1, log-likelihood eq. 2, gradients
eqs. 8-10.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "HawkesError", "lib", "library_path", "workspace_bytes", "loglik", "loglik_grad",
    "intensity", "loglik_batched", "loglik_grad_batched", "sequential_loglik_grad",
    "check_inputs", "HawkesLogLik", "hawkes_loglik", "BETA_SHARED", "BETA_PER_TARGET", "AdamMLE",
    "Batch", "BatchedGraph", "batched_workspace_bytes", "loglik_grad_noalloc", "simulate", "simulate_n",
    "stationary_rate", "philox4x64_10",
]

BETA_SHARED = 0
BETA_PER_TARGET = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libhawkes.so")
_lib = None

_STATUS = {0: "ok", 1: "invalid argument", 2: "workspace missing or too small", 3: "device error",
           4: "unsupported request"}


class HawkesError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: status {status} ({_STATUS.get(status, 'unknown')})")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("beta_mode", ctypes.c_int32), ("chunk_log2", ctypes.c_int32), ("T", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("dense_cols", ctypes.c_int32), ("dense_ranges", ctypes.c_int32), ("item_log2", ctypes.c_int32),
                ("dense_rows", ctypes.c_int32)]


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("floor_mu", ctypes.c_float), ("floor_beta", ctypes.c_float),
                ("lambda1", ctypes.c_float), ("h", ctypes.c_float), ("flags", ctypes.c_uint32)]


def library_path() -> str:
    return _LIBPATH


def lib():
    """Load libhawkes.so (built in-tree).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"{_LIBPATH} is missing: build it with paper_2604_01342_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(_LIBPATH)
    vp, sz, i32, i64, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER(_Problem)
    L.hawkes_status_string.argtypes = [ctypes.c_int]
    L.hawkes_status_string.restype = ctypes.c_char_p
    L.hawkes_version.restype = ctypes.c_int
    L.hawkes_workspace_bytes.argtypes = [P, ctypes.c_int]
    L.hawkes_workspace_bytes.restype = sz
    L.hawkes_loglik.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_loglik_grad.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_loglik_grad_support.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_loglik_grad_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.hawkes_intensity.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_sequential_loglik_grad.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_check_inputs.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
    L.hawkes_batched_workspace_bytes.argtypes = [i32, i64, i32, ctypes.c_int]
    L.hawkes_batched_workspace_bytes.restype = sz
    L.hawkes_loglik_batched.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.hawkes_loglik_grad_batched.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                             sz, vp]
    L.hawkes_set_tuning.argtypes = [ctypes.POINTER(_Tuning)]
    L.hawkes_get_tuning.argtypes = [ctypes.POINTER(_Tuning)]
    L.hawkes_set_tuning.restype = ctypes.c_int
    L.hawkes_get_tuning.restype = ctypes.c_int
    L.hawkes_timing_enable.argtypes = [ctypes.c_int]
    L.hawkes_timing_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for f in ("hawkes_timing_enable", "hawkes_timing_reset", "hawkes_timing_read"):
        getattr(L, f).restype = ctypes.c_int
    L.hawkes_simulate_workspace_bytes.argtypes = [i32, i32, i64]
    L.hawkes_simulate_workspace_bytes.restype = sz
    L.hawkes_simulate.argtypes = [i32, i32, i32, vp, vp, vp, d, ctypes.c_uint64, i64, vp, vp,
                                  ctypes.POINTER(ctypes.c_int64), vp, sz, vp]
    L.hawkes_simulate.restype = ctypes.c_int
    L.hawkes_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64)]
    L.hawkes_philox4x64_10.restype = None
    L.hawkes_adam_state_bytes.argtypes = [P]
    L.hawkes_adam_state_bytes.restype = sz
    L.hawkes_adam_init.argtypes = [P, vp, sz, vp]
    L.hawkes_adam_step.argtypes = [P, vp, vp, vp, vp, vp, ctypes.POINTER(_Adam), vp, sz, vp, vp, vp, vp, vp, sz, vp]
    for f in ("hawkes_loglik", "hawkes_loglik_grad", "hawkes_loglik_grad_support", "hawkes_loglik_grad_noalloc",
              "hawkes_intensity", "hawkes_sequential_loglik_grad",
              "hawkes_check_inputs", "hawkes_loglik_batched", "hawkes_loglik_grad_batched", "hawkes_adam_init",
              "hawkes_adam_step"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check(fn, status):
    if status != 0:
        raise HawkesError(fn, status)


_ws_cache: dict = {}


def _workspace(dev, nbytes: int) -> torch.Tensor:
    """Reusable, 256-byte aligned device scratch (grown on demand)."""
    key = (dev.type, dev.index)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes + 256:
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        _ws_cache[key] = buf
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def _prep(t, m, mu, alpha, beta):
    dev = mu.device
    if dev.type != "cuda":
        raise ValueError("tensors must be on a GPU device")
    t = t.to(device=dev, dtype=torch.float64).contiguous()
    m = m.to(device=dev, dtype=torch.int32).contiguous()
    mu = mu.detach().to(dtype=torch.float32).contiguous()
    alpha = alpha.detach().to(dtype=torch.float32).contiguous()
    beta = beta.detach().to(device=dev, dtype=torch.float32).reshape(-1).contiguous()
    M = mu.numel()
    if alpha.numel() == 0 or alpha.numel() % (M * M):
        raise ValueError("alpha must be M x M or K x M x M")
    if t.numel() != m.numel():
        raise ValueError("t and marks differ in length")
    return dev, t, m, mu, alpha, beta


def _kernels(mu, alpha) -> int:
    """Number of decay kernels K from alpha's size (K x M x M)."""
    return alpha.numel() // (mu.numel() ** 2)


def _problem(t, mu, beta, T, chunk_log2, alpha=None):
    """K decay kernels (alpha K x M x M) share a decay each (beta[K]); with
    K = 1, beta[M] selects one decay per target node."""
    M = mu.numel()
    K = 1 if alpha is None else _kernels(mu, alpha)
    if K > 1:
        if beta.numel() != K:
            raise ValueError("with K kernels beta must have K entries")
        mode = BETA_SHARED
    else:
        mode = BETA_SHARED if beta.numel() == 1 else BETA_PER_TARGET
        if mode == BETA_PER_TARGET and beta.numel() != M:
            raise ValueError("beta must have 1 or M entries")
    return _Problem(t.numel(), M, K, mode, int(chunk_log2), float(T))


def _gshape(mu, alpha):
    """Shape of dL/dalpha: (M, M), or (K, M, M) with several kernels."""
    M = mu.numel()
    K = _kernels(mu, alpha)
    return (M, M) if K == 1 else (K, M, M)


def set_tuning(dense_cols: int = 0, dense_ranges: int = 0, item_log2: int = 0, dense_rows: int = 0) -> None:
    """Process-wide launch tuning (hawkes_set_tuning): 0 keeps the library's
    rule.  dense_cols in {64, 128, 256}, dense_ranges a power of two up to
    4096, item_log2 in 4..16, dense_rows in {16, 32}.  Results agree to
    rounding whatever the values."""
    t = _Tuning(int(dense_cols), int(dense_ranges), int(item_log2), int(dense_rows))
    _check("hawkes_set_tuning", lib().hawkes_set_tuning(ctypes.byref(t)))


def get_tuning() -> dict:
    """The current process-wide launch tuning (hawkes_get_tuning)."""
    t = _Tuning()
    _check("hawkes_get_tuning", lib().hawkes_get_tuning(ctypes.byref(t)))
    return {"dense_cols": t.dense_cols, "dense_ranges": t.dense_ranges, "item_log2": t.item_log2,
            "dense_rows": t.dense_rows}


def workspace_bytes(n: int, M: int, per_target: bool = False, grad: bool = True, chunk_log2: int = 0,
                    K: int = 1) -> int:
    p = _Problem(n, M, K, BETA_PER_TARGET if per_target else BETA_SHARED, chunk_log2, 1.0)
    return int(lib().hawkes_workspace_bytes(ctypes.byref(p), int(grad)))


def loglik(t, m, mu, alpha, beta, T, chunk_log2: int = 0) -> torch.Tensor:
    """Log-likelihood (eq. 2) as a float64 0-d device tensor."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, chunk_log2, alpha)
    L = lib()
    nb = L.hawkes_workspace_bytes(ctypes.byref(p), 0)
    ws = _workspace(dev, nb)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    _check("hawkes_loglik", L.hawkes_loglik(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu), _ptr(alpha), _ptr(beta),
                                            _ptr(out), _ptr(ws), nb, _stream(dev)))
    return out[0]


def loglik_grad(t, m, mu, alpha, beta, T, chunk_log2: int = 0, support: bool = False):
    """(L, dL/dmu [M], dL/dalpha [M, M], dL/dbeta [1] or [M]) as float64 device tensors.
    support=True: dL/dalpha only at alpha's nonzeros, 0 elsewhere
    (hawkes_loglik_grad_support)."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, chunk_log2, alpha)
    L = lib()
    nb = L.hawkes_workspace_bytes(ctypes.byref(p), 1)
    ws = _workspace(dev, nb)
    M = mu.numel()
    out = torch.empty(1, dtype=torch.float64, device=dev)
    gmu = torch.empty(M, dtype=torch.float64, device=dev)
    ga = torch.empty(_gshape(mu, alpha), dtype=torch.float64, device=dev)
    gb = torch.empty(beta.numel(), dtype=torch.float64, device=dev)
    name = "hawkes_loglik_grad_support" if support else "hawkes_loglik_grad"
    _check(name, getattr(L, name)(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu), _ptr(alpha), _ptr(beta), _ptr(out),
                                  _ptr(gmu), _ptr(ga), _ptr(gb), _ptr(ws), nb, _stream(dev)))
    return out[0], gmu, ga, gb


NOALLOC_SCRATCH_BYTES = 64 << 20   # HAWKES_NOALLOC_SCRATCH_BYTES


def loglik_grad_noalloc(t, m, mu, alpha, beta, T, chunk_log2: int = 0, out=None):
    """As loglik_grad, through hawkes_loglik_grad_noalloc: the library takes
    its workspace from its fixed per-device scratch (problems whose workspace
    exceeds NOALLOC_SCRATCH_BYTES are refused).  ``out``: preallocated
    (loglik[1], g_mu[M], g_alpha[M, M], g_beta) float64 tensors, so that the
    call allocates nothing on this side either."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, chunk_log2, alpha)
    M = mu.numel()
    if out is None:
        out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(M, dtype=torch.float64, device=dev),
               torch.empty(_gshape(mu, alpha), dtype=torch.float64, device=dev),
               torch.empty(beta.numel(), dtype=torch.float64, device=dev))
    ll, gmu, ga, gb = out
    _check("hawkes_loglik_grad_noalloc",
           lib().hawkes_loglik_grad_noalloc(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu), _ptr(alpha), _ptr(beta),
                                            _ptr(ll), _ptr(gmu), _ptr(ga), _ptr(gb), _stream(dev)))
    return ll[0], gmu, ga, gb


def intensity(t, m, mu, alpha, beta, T, chunk_log2: int = 0) -> torch.Tensor:
    """lambda_{m_i}(t_i) for every event (eq. 1), float32."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, chunk_log2, alpha)
    L = lib()
    nb = L.hawkes_workspace_bytes(ctypes.byref(p), 0)
    ws = _workspace(dev, nb)
    lam = torch.empty(t.numel(), dtype=torch.float32, device=dev)
    _check("hawkes_intensity", L.hawkes_intensity(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu), _ptr(alpha),
                                                  _ptr(beta), _ptr(lam), _ptr(ws), nb, _stream(dev)))
    return lam


def sequential_loglik_grad(t, m, mu, alpha, beta, T):
    """Same outputs as loglik_grad from the one-workgroup sequential baseline kernel."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, 0, alpha)
    L = lib()
    M = mu.numel()
    nb = M * M * 8 + 512
    ws = _workspace(dev, nb)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    gmu = torch.empty(M, dtype=torch.float64, device=dev)
    ga = torch.empty(M, M, dtype=torch.float64, device=dev)
    gb = torch.empty(1, dtype=torch.float64, device=dev)
    _check("hawkes_sequential_loglik_grad",
           L.hawkes_sequential_loglik_grad(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu), _ptr(alpha), _ptr(beta),
                                           _ptr(out), _ptr(gmu), _ptr(ga), _ptr(gb), _ptr(ws), nb, _stream(dev)))
    return out[0], gmu, ga, gb


def philox4x64_10(ctr, key) -> list:
    """The simulator's counter-based generator (Philox4x64-10) evaluated on
    the host: four 64-bit outputs for a 4-word counter and 2-word key."""
    c = (ctypes.c_uint64 * 4)(*[int(x) & (2 ** 64 - 1) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) & (2 ** 64 - 1) for x in key])
    out = (ctypes.c_uint64 * 4)()
    lib().hawkes_philox4x64_10(c, k, out)
    return [int(x) for x in out]


def stationary_rate(mu, alpha) -> float:
    """Expected events per unit time of the stationary process,
    1^T (I - sum_k alpha_k)^{-1} mu (host arithmetic on the parameters, for
    sizing simulations; rho(sum_k alpha_k) < 1 is assumed)."""
    import numpy as np
    mu = np.asarray(mu.detach().cpu() if isinstance(mu, torch.Tensor) else mu, dtype=np.float64).reshape(-1)
    a = np.asarray(alpha.detach().cpu() if isinstance(alpha, torch.Tensor) else alpha, dtype=np.float64)
    M = mu.shape[0]
    A = a.reshape(-1, M, M).sum(axis=0)
    return float(np.linalg.solve(np.eye(M) - A, mu).sum())


def simulate(mu, alpha, beta, T0: float, seed: int, capacity: int | None = None):
    """Events of the process on [0, T0] by its branching representation, on
    the GPU (hawkes_simulate): (t float64, marks int32) device tensors sorted
    by time.  alpha M x M or K x M x M; beta [K] (a decay per kernel) or, with
    K = 1, [M] (a decay per target node).  The result depends only on seed and
    the parameters.  capacity: event slots to reserve (default: 1.25 times the
    stationary expectation plus a margin; grown and retried if exceeded)."""
    dev = mu.device
    if dev.type != "cuda":
        raise ValueError("tensors must be on a GPU device")
    mu = mu.detach().to(dtype=torch.float32).contiguous()
    alpha = alpha.detach().to(dtype=torch.float32).contiguous()
    beta = beta.detach().to(device=dev, dtype=torch.float32).reshape(-1).contiguous()
    M = mu.numel()
    K = _kernels(mu, alpha)
    if K > 1 and beta.numel() != K:
        raise ValueError("with K kernels beta must have K entries")
    mode = BETA_PER_TARGET if K == 1 and beta.numel() == M and M > 1 else BETA_SHARED
    if mode == BETA_SHARED and beta.numel() != K:
        raise ValueError("beta must have K or (with K = 1) M entries")
    if capacity is None:
        capacity = int(1.25 * T0 * stationary_rate(mu, alpha)) + 10_000
    L = lib()
    while True:
        capacity = max(int(capacity), 1)
        nb = int(L.hawkes_simulate_workspace_bytes(M, K, capacity))
        if nb == 0:
            raise HawkesError("hawkes_simulate_workspace_bytes", 1)
        ws = _aligned(dev, nb)
        t = torch.empty(capacity, dtype=torch.float64, device=dev)
        m = torch.empty(capacity, dtype=torch.int32, device=dev)
        n = ctypes.c_int64(0)
        st = L.hawkes_simulate(M, K, mode, _ptr(mu), _ptr(alpha), _ptr(beta), float(T0), ctypes.c_uint64(seed),
                               capacity, _ptr(t), _ptr(m), ctypes.byref(n), _ptr(ws), nb, _stream(dev))
        if st == 2 and n.value > capacity:
            capacity = max(2 * capacity, int(1.25 * n.value))
            continue
        _check("hawkes_simulate", st)
        return t[:n.value], m[:n.value]


def simulate_n(mu, alpha, beta, n: int, seed: int):
    """The first n events of a simulated sequence and T = t_n (the window end
    of an event-count-stopped sample): T0 = 1.2 n / stationary rate, enlarged
    1.5 times (same seed) until the window holds n events."""
    T0 = 1.2 * n / stationary_rate(mu, alpha)
    while True:
        t, m = simulate(mu, alpha, beta, T0, seed)
        if t.numel() >= n:
            t, m = t[:n].clone(), m[:n].clone()
            return t, m, float(t[-1].item()) if n else 0.0
        T0 *= 1.5


TIMING_KERNELS = {0: "dense_dalpha", 1: "forward", 2: "segment_aggregate", 3: "segment_scan",
                  4: "small_compute", 5: "small_scan", 6: "bucket", 7: "dense_checkpoints"}


def timing_enable(on: bool = True, kernels=None) -> None:
    """Record hipEvents around the library's main kernels (diagnostics):
    every kernel, or only the ids in ``kernels`` (see TIMING_KERNELS)."""
    if not on:
        v = 0
    elif kernels is None:
        v = -1
    else:
        v = 0
        for k in kernels:
            v |= 1 << int(k)
    _check("hawkes_timing_enable", lib().hawkes_timing_enable(v))


def timing_reset() -> None:
    _check("hawkes_timing_reset", lib().hawkes_timing_reset())


def timing_read() -> dict:
    """{kernel name: (total_ms, launches)} accumulated since the last reset (waits on the events)."""
    out = {}
    for k, name in TIMING_KERNELS.items():
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check("hawkes_timing_read", lib().hawkes_timing_read(k, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (ms.value, n.value)
    return out


def check_inputs(t, m, mu, alpha, beta, T) -> int:
    """Device-side precondition check; returns the status bit mask (0 = valid).  Synchronises."""
    dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    p = _problem(t, mu, beta, T, 0, alpha)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    _check("hawkes_check_inputs", lib().hawkes_check_inputs(ctypes.byref(p), _ptr(t), _ptr(m), _ptr(mu),
                                                            _ptr(alpha), _ptr(beta), _ptr(st), _stream(dev)))
    return int(st.item())


@dataclass
class Batch:
    """Device-resident packed batch of S sequences (see hawkes.h)."""
    ev_off: torch.Tensor
    m_s: torch.Tensor
    T_s: torch.Tensor
    t: torch.Tensor
    m: torch.Tensor
    mu: torch.Tensor
    alpha: torch.Tensor
    beta: torch.Tensor
    max_m: int

    @property
    def S(self) -> int:
        return int(self.m_s.numel())

    @classmethod
    def from_numpy(cls, bw, device="cuda"):
        d = torch.device(device)
        return cls(torch.as_tensor(bw.ev_off, dtype=torch.int64, device=d),
                   torch.as_tensor(bw.m_s, dtype=torch.int32, device=d),
                   torch.as_tensor(bw.T_s, dtype=torch.float64, device=d),
                   torch.as_tensor(bw.t, dtype=torch.float64, device=d),
                   torch.as_tensor(bw.m, dtype=torch.int32, device=d),
                   torch.as_tensor(bw.mu, dtype=torch.float32, device=d),
                   torch.as_tensor(bw.alpha, dtype=torch.float32, device=d),
                   torch.as_tensor(bw.beta, dtype=torch.float32, device=d),
                   int(bw.m_s.max()))


def batched_workspace_bytes(b: Batch, grad: bool = True) -> int:
    """Workspace bytes of a batched call on ``b`` (hawkes_batched_workspace_bytes)."""
    nb = int(lib().hawkes_batched_workspace_bytes(b.S, b.t.numel(), b.max_m, int(grad)))
    if nb == 0:
        raise HawkesError("hawkes_batched_workspace_bytes", 1)
    return nb


def _batched(b: Batch, grad: bool, out=None, ws=None):
    """ws: a caller-owned workspace (256-byte aligned, at least the queried
    size) instead of the module's shared one."""
    dev = b.t.device
    L = lib()
    n_total = b.t.numel()
    nb = batched_workspace_bytes(b, grad)
    if ws is None:
        ws = _workspace(dev, nb)
    elif ws.numel() < nb or ws.data_ptr() % 256:
        raise ValueError("workspace too small or not 256-byte aligned")
    if out is None:
        out = (torch.empty(b.S, dtype=torch.float64, device=dev),
               torch.empty(b.mu.numel(), dtype=torch.float64, device=dev) if grad else None,
               torch.empty(b.alpha.numel(), dtype=torch.float64, device=dev) if grad else None,
               torch.empty(b.S, dtype=torch.float64, device=dev) if grad else None)
    ll, gmu, ga, gb = out
    if grad:
        st = L.hawkes_loglik_grad_batched(b.S, n_total, b.max_m, _ptr(b.ev_off), _ptr(b.m_s), _ptr(b.T_s),
                                          _ptr(b.t), _ptr(b.m), _ptr(b.mu), _ptr(b.alpha), _ptr(b.beta),
                                          _ptr(ll), _ptr(gmu), _ptr(ga), _ptr(gb), _ptr(ws), nb, _stream(dev))
        _check("hawkes_loglik_grad_batched", st)
        return ll, gmu, ga, gb
    st = L.hawkes_loglik_batched(b.S, n_total, b.max_m, _ptr(b.ev_off), _ptr(b.m_s), _ptr(b.T_s), _ptr(b.t),
                                 _ptr(b.m), _ptr(b.mu), _ptr(b.alpha), _ptr(b.beta), _ptr(ll), _ptr(ws), nb,
                                 _stream(dev))
    _check("hawkes_loglik_batched", st)
    return ll


def loglik_batched(b: Batch) -> torch.Tensor:
    """Per-sequence log-likelihoods [S] (float64)."""
    return _batched(b, False)


def loglik_grad_batched(b: Batch, out=None):
    """(loglik[S], g_mu packed like mu, g_alpha packed like alpha, g_beta[S])."""
    return _batched(b, True, out)


class BatchedGraph:
    """One batched loglik+grad call recorded in a HIP graph, then replayed.

    Every replay reads the batch's device arrays in place (new values of the
    same shapes written into them are picked up) and writes the same output
    tensors, ``out``.  The graph owns its workspace (the captured kernels
    point into it), so later calls of any size elsewhere cannot move it.  The
    launch tuning in effect at capture is baked in: capture again after
    changing it."""

    def __init__(self, b: Batch):
        if b.max_m > 8:
            raise ValueError("a batch with more than 8 nodes in a sequence synchronises with the host "
                             "(hawkes_loglik_grad_batched) and cannot be captured in a graph")
        self.b = b
        dev = b.t.device
        self.out = (torch.empty(b.S, dtype=torch.float64, device=dev),
                    torch.empty(b.mu.numel(), dtype=torch.float64, device=dev),
                    torch.empty(b.alpha.numel(), dtype=torch.float64, device=dev),
                    torch.empty(b.S, dtype=torch.float64, device=dev))
        self.ws = _aligned(dev, batched_workspace_bytes(b, True))
        # an eager call first: loads the library and sets kernel attributes,
        # so that nothing allocates during capture
        _batched(b, True, self.out, self.ws)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            _batched(b, True, self.out, self.ws)

    def replay(self):
        """(loglik[S], g_mu, g_alpha, g_beta[S]) of the batch's current values."""
        self.graph.replay()
        return self.out


class HawkesLogLik(torch.autograd.Function):
    """L(mu, alpha, beta) for a fixed event sequence.  When any parameter
    needs a gradient, forward runs the fused log-likelihood + gradient call
    (forward-mode states with chunk-boundary carries, no per-event storage);
    backward scales the stored gradient by the incoming scalar."""

    @staticmethod
    def forward(ctx, mu, alpha, beta, t, m, T, chunk_log2=0):
        need = any(ctx.needs_input_grad[:3])
        if need:
            L, gmu, ga, gb = loglik_grad(t, m, mu, alpha, beta, T, chunk_log2)
            ctx.save_for_backward(gmu, ga, gb)
        else:
            L = loglik(t, m, mu, alpha, beta, T, chunk_log2)
        ctx.shapes = (mu.shape, alpha.shape, beta.shape)
        ctx.dtypes = (mu.dtype, alpha.dtype, beta.dtype)
        return L

    @staticmethod
    def backward(ctx, gL):
        gmu, ga, gb = ctx.saved_tensors
        (smu, sa, sb), (dmu, da, db) = ctx.shapes, ctx.dtypes
        return ((gL * gmu).reshape(smu).to(dmu), (gL * ga).reshape(sa).to(da), (gL * gb).reshape(sb).to(db),
                None, None, None, None)


def hawkes_loglik(t, m, mu, alpha, beta, T, chunk_log2: int = 0) -> torch.Tensor:
    """Differentiable log-likelihood w.r.t. (mu, alpha, beta)."""
    return HawkesLogLik.apply(mu, alpha, beta, t, m, T, chunk_log2)


def _aligned(dev, nbytes: int) -> torch.Tensor:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


class AdamMLE:
    """Maximum-likelihood fit by projected Adam on the per-event negative
    log-likelihood plus the hinge-l1 sparsity penalty lambda1 * sum over
    off-diagonal alpha_pq < h of alpha_pq (lambda1 = 0: no penalty; log_mu,
    log_beta, log_alpha: steps on the logarithms), one
    hawkes_adam_step call per step (evaluation, gradient and update on the
    GPU, no host synchronisation).  Owns float32 copies of
    the parameters (updated in place), its workspace, the optimizer state and
    the last step's outputs.  capture() records one step in a HIP graph;
    replay() runs it again (each replay is one more Adam step)."""

    def __init__(self, t, m, mu, alpha, beta, T, lr=0.05, betas=(0.9, 0.999), eps=1e-8, floor_mu=1e-6,
                 floor_beta=1e-6, chunk_log2: int = 0, lambda1: float = 0.0, h: float = 0.05,
                 log_mu: bool = False, log_beta: bool = False, log_alpha: bool = False):
        dev, t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
        self.dev, self.t, self.m = dev, t, m
        self.mu, self.alpha, self.beta = mu.clone(), alpha.clone(), beta.clone()
        self.p = _problem(t, self.mu, self.beta, T, chunk_log2, self.alpha)
        L = lib()
        self.ws_bytes = int(L.hawkes_workspace_bytes(ctypes.byref(self.p), 1))
        self.ws = _aligned(dev, self.ws_bytes)
        self.state_bytes = int(L.hawkes_adam_state_bytes(ctypes.byref(self.p)))
        if self.state_bytes == 0:
            raise ValueError("invalid problem for the Adam state")
        self.state = _aligned(dev, self.state_bytes)
        self.cfg = _Adam(lr, betas[0], betas[1], eps, floor_mu, floor_beta, lambda1, h,
                         (1 if log_mu else 0) | (2 if log_beta else 0) | (4 if log_alpha else 0))
        M = self.mu.numel()
        self.loglik = torch.empty(1, dtype=torch.float64, device=dev)
        self.g_mu = torch.empty(M, dtype=torch.float64, device=dev)
        self.g_alpha = torch.empty(_gshape(self.mu, self.alpha), dtype=torch.float64, device=dev)
        self.g_beta = torch.empty(self.beta.numel(), dtype=torch.float64, device=dev)
        self.graph = None
        _check("hawkes_adam_init", L.hawkes_adam_init(ctypes.byref(self.p), _ptr(self.state), self.state_bytes,
                                                      _stream(dev)))

    def step(self):
        """One evaluation + Adam step on the current stream; returns L at the
        parameters before the step (device tensor)."""
        L = lib()
        _check("hawkes_adam_step",
               L.hawkes_adam_step(ctypes.byref(self.p), _ptr(self.t), _ptr(self.m), _ptr(self.mu), _ptr(self.alpha),
                                  _ptr(self.beta), ctypes.byref(self.cfg), _ptr(self.state), self.state_bytes,
                                  _ptr(self.loglik), _ptr(self.g_mu), _ptr(self.g_alpha), _ptr(self.g_beta),
                                  _ptr(self.ws), self.ws_bytes, _stream(self.dev)))
        return self.loglik[0]

    def capture(self):
        """Record one step into a HIP graph (nothing runs during capture)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.loglik[0]
