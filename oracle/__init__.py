"""ctypes binding of the FP64 CPU oracle (hawkes_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hawkes_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        sig = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _d, _i32,
               _d, _d, _d, _d, _d, _d, _d]
        for name in ("oracle_brute", "oracle_forward"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.oracle_adjoint.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _d, _i32,
                                     _d, _d, _d, _d, _d, _d, _d]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_intensity_at.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _i32,
                                          _d, _d, _d, ctypes.c_int64, _i64, _d]
        L.oracle_intensity_at.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ct) if a is not None else None


def _prep(t, m, mu, alpha, beta):
    t = np.ascontiguousarray(t, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.int32)
    mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
    return t, m, mu, alpha, beta


def brute(t, m, mu, alpha, beta, T, grad=True):
    """Definition (eqs. 1, 2, 8-10) as O(N^2) sums.  alpha [K,M,M] or [M,M];
    beta [K,M] (per kernel and target), [K] (shared) or [M] with K=1 per target.
    Returns (L, g_mu, g_alpha, g_beta[K,M])."""
    t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    M = mu.shape[0]
    a3 = alpha.reshape(-1, M, M)
    K = a3.shape[0]
    if beta.shape[0] == K:
        b2 = np.repeat(beta.reshape(K, 1), M, axis=1)
    elif beta.shape[0] == K * M:
        b2 = beta.reshape(K, M)
    else:
        raise ValueError("beta shape")
    b2 = np.ascontiguousarray(b2)
    L = np.zeros(1)
    gmu = np.zeros(M) if grad else None
    ga = np.zeros((K, M, M)) if grad else None
    gb = np.zeros((K, M)) if grad else None
    rc = lib().oracle_brute(t.shape[0], M, K, float(T), _p(t, _d), _p(m, _i32), _p(mu, _d),
                            _p(np.ascontiguousarray(a3), _d), _p(b2, _d), _p(L, _d),
                            _p(gmu, _d), _p(ga, _d), _p(gb, _d))
    if rc != 0:
        raise ValueError("oracle_brute rejected its arguments")
    return (float(L[0]), gmu, ga, gb) if grad else float(L[0])


def forward(t, m, mu, alpha, beta, T, grad=True):
    """Sequential forward-mode recurrence, decay shared per kernel.
    alpha [K,M,M] or [M,M], beta [K].  Returns (L, g_mu[M], g_alpha[K,M,M], g_beta[K])."""
    t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    M = mu.shape[0]
    a3 = np.ascontiguousarray(alpha.reshape(-1, M, M))
    K = a3.shape[0]
    if beta.shape[0] != K:
        raise ValueError("forward() needs one decay per kernel")
    L = np.zeros(1)
    gmu = np.zeros(M) if grad else None
    ga = np.zeros((K, M, M)) if grad else None
    gb = np.zeros(K) if grad else None
    rc = lib().oracle_forward(t.shape[0], M, K, float(T), _p(t, _d), _p(m, _i32), _p(mu, _d),
                              _p(a3, _d), _p(beta, _d), _p(L, _d), _p(gmu, _d), _p(ga, _d),
                              _p(gb, _d))
    if rc != 0:
        raise ValueError("oracle_forward rejected its arguments")
    return (float(L[0]), gmu, ga, gb) if grad else float(L[0])


def adjoint(t, m, mu, alpha, beta, T, grad=True):
    """Reverse-mode pass, one kernel, decay per target (beta [M]).
    Returns (L, g_mu[M], g_alpha[M,M], g_beta[M])."""
    t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    M = mu.shape[0]
    a2 = np.ascontiguousarray(alpha.reshape(M, M))
    if beta.shape[0] == 1 and M > 1:
        beta = np.full(M, beta[0])
    L = np.zeros(1)
    gmu = np.zeros(M) if grad else None
    ga = np.zeros((M, M)) if grad else None
    gb = np.zeros(M) if grad else None
    rc = lib().oracle_adjoint(t.shape[0], M, float(T), _p(t, _d), _p(m, _i32), _p(mu, _d),
                              _p(a2, _d), _p(beta, _d), _p(L, _d), _p(gmu, _d), _p(ga, _d),
                              _p(gb, _d))
    if rc != 0:
        raise ValueError("oracle_adjoint rejected its arguments")
    return (float(L[0]), gmu, ga, gb) if grad else float(L[0])


def intensity_at(t, m, mu, alpha, beta, idx):
    """lambda_{m_i}(t_i) by the definition at the given indices.  beta as in brute()."""
    t, m, mu, alpha, beta = _prep(t, m, mu, alpha, beta)
    M = mu.shape[0]
    a3 = np.ascontiguousarray(alpha.reshape(-1, M, M))
    K = a3.shape[0]
    if beta.shape[0] == K:
        b2 = np.repeat(beta.reshape(K, 1), M, axis=1)
    else:
        b2 = beta.reshape(K, M)
    b2 = np.ascontiguousarray(b2)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0])
    rc = lib().oracle_intensity_at(t.shape[0], M, K, _p(t, _d), _p(m, _i32), _p(mu, _d),
                                   _p(a3, _d), _p(b2, _d), idx.shape[0], _p(idx, _i64),
                                   _p(out, _d))
    if rc != 0:
        raise ValueError("oracle_intensity_at rejected its arguments")
    return out


def addend_scales(t, m, mu, alpha, beta, T, grads):
    """Scales for the addend-scaled gradient error at the generating point.

    Each gradient block is a difference of two nonnegative sums (eqs. 8-10):
    dL/dmu_p = S_p - T, dL/dalpha_pq = G_pq - C_q, dL/dbeta = G_beta - E with
    C_q = sum_{j: m_j = q} (1 - e^{-beta (T - t_j)}) and
    E = sum_j colsum_{m_j} (T - t_j) e^{-beta (T - t_j)} (shared decay, one
    kernel).  Given the oracle's gradients, the positive parts follow as
    gradient + negative part; the returned scales are the norms of
    |positive| + |negative| per block, so that error / scale measures the
    error against the size of the addends rather than against their near-
    cancelling difference."""
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.int64)
    M = np.asarray(mu).shape[0]
    a = np.asarray(alpha, dtype=np.float64).reshape(M, M)
    b = float(np.asarray(beta, dtype=np.float64).ravel()[0])
    g_mu, g_a, g_b = (np.asarray(x, dtype=np.float64) for x in grads)
    g_a = g_a.reshape(M, M)
    x = b * (T - t)
    C = np.bincount(m, weights=-np.expm1(-x), minlength=M)
    colsum = a.sum(axis=0)
    E = float(np.sum(colsum[m] * (T - t) * np.exp(-x)))
    s_mu = np.linalg.norm(np.abs(g_mu + T) + T)
    s_a = np.linalg.norm(np.abs(g_a + C[None, :]) + C[None, :])
    s_b = abs(float(np.ravel(g_b)[0]) + E) + E
    return float(s_mu), float(s_a), float(s_b)


def sparsity_penalty(alpha, lam, h):
    """Hinge-l1 sparsity penalty of the training objective (section
    "Background": the per-event NLL plus lam times the sum of alpha's
    off-diagonal entries that lie below the hinge point h) and its gradient
    with respect to alpha: lam at those entries, zero on the diagonal and at
    or above h (the indicator's jump at h is ignored, as a gradient step
    does).  The comparison alpha < h is made on the values as given, so a
    float32 alpha and a float32 h decide as the library does.  Returns
    (value, grad), grad in float64 and shaped like alpha (M x M)."""
    a = np.asarray(alpha)
    M = a.shape[0]
    value = 0.0
    grad = np.zeros((M, M), dtype=np.float64)
    for p in range(M):
        for q in range(M):
            if p != q and a[p, q] < h:
                value += float(a[p, q])
                grad[p, q] = lam
    return lam * value, grad
