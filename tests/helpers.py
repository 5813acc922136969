"""Shared test helpers: problem generators and error metrics (no model arithmetic)."""
import numpy as np


def rel_err(a, b):
    """Normwise relative error ||a - b|| / ||b|| (Frobenius for matrices)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def scalar_rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def rand_problem(seed, n, M, per_target=False, ties=False, density=1.0, rate=1.0, rho=0.5):
    """Random sorted event sequence with float32 parameters (as the GPU sees them)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    if ties and n > 3:
        gaps[rng.random(n) < 0.15] = 0.0
    t = np.cumsum(gaps)
    m = rng.integers(0, M, size=n).astype(np.int32)
    mu = rng.uniform(0.05, 0.5, size=M).astype(np.float32)
    a = rng.uniform(0.0, 1.0, size=(M, M))
    if density < 1.0:
        a *= rng.random((M, M)) < density
    s = a.sum(axis=0).max()
    alpha = (a * (rho / s if s > 0 else 1.0)).astype(np.float32)
    beta = (rng.uniform(0.5, 2.0, size=M) if per_target else rng.uniform(0.5, 2.0, size=1)).astype(np.float32)
    T = float(t[-1] + rng.uniform(0.0, 1.0)) if n else 1.5
    return t, m, mu, alpha, beta, T
