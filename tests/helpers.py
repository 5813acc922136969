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


class PackedBatch:
    """Packed arrays of S sequences in the batched ABI's layout (see hawkes.h)."""

    def __init__(self, ev_off, m_s, T_s, t, m, mu, alpha, beta):
        self.ev_off, self.m_s, self.T_s, self.t, self.m = ev_off, m_s, T_s, t, m
        self.mu, self.alpha, self.beta = mu, alpha, beta
        self.S = len(m_s)
        self.mu_off = np.concatenate([[0], np.cumsum(m_s)]).astype(np.int64)
        self.a_off = np.concatenate([[0], np.cumsum(m_s.astype(np.int64) ** 2)]).astype(np.int64)

    def seq(self, s):
        """(t, marks, mu, alpha [M, M], beta [1], T) of sequence s."""
        M = int(self.m_s[s])
        e0, e1 = int(self.ev_off[s]), int(self.ev_off[s + 1])
        return (self.t[e0:e1], self.m[e0:e1], self.mu[self.mu_off[s]:self.mu_off[s + 1]],
                self.alpha[self.a_off[s]:self.a_off[s + 1]].reshape(M, M), self.beta[s:s + 1], float(self.T_s[s]))


def rand_batch(seed, S, m_choices, lo=1, hi=10_000, n_empty=0, rate=2.0):
    """S random sorted sequences with node counts drawn from m_choices and
    lengths log-uniform in [lo, hi] (the first n_empty sequences are empty)."""
    rng = np.random.default_rng(seed)
    m_s = rng.choice(np.asarray(m_choices), size=S).astype(np.int32)
    lens = np.exp(rng.uniform(np.log(lo), np.log(hi), size=S)).round().astype(np.int64)
    lens[:n_empty] = 0
    parts = [rand_problem(int(rng.integers(1 << 30)), int(lens[s]), int(m_s[s]), rate=rate) for s in range(S)]
    ev_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cat = lambda k, dt: (np.concatenate([np.ravel(p[k]) for p in parts]).astype(dt) if S else np.zeros(0, dt))
    return PackedBatch(ev_off, m_s, np.array([p[5] for p in parts]), cat(0, np.float64), cat(1, np.int32),
                       cat(2, np.float32), cat(3, np.float32), cat(4, np.float32))
