"""Seeded synthetic Hawkes workloads.

Input generation only: this module simulates event sequences and draws
parameters.  It computes neither the log-likelihood nor its gradient, and it
is shared by the tests (which feed its output to both the CPU oracle and the
GPU library) and by the benchmark.

Conventions (paper, Background, eq. 1): alpha[p, q] is the excitation of
target p by a source event of node q, and the kernel beta*exp(-beta*x) is
normalised, so alpha is the branching matrix; "rescaled to spectral radius rho"
means rho(alpha) = rho < 1.  Workloads stop after N events and set the
observation window end T to the N-th event time.

The five named workloads mirror the sizes and parameter distributions used
for the throughput study:
  c1  M=1, N=10,000, mu=0.5, alpha=0.5, beta=1, Ogata thinning
  c2  M=16, N=1,000,000, mu~U[0.05,0.2], dense alpha U[0,1] -> rho 0.7, beta=1
  c3  4096 sequences, M=8, lengths log-uniform in [100, 100000],
      mu~U[0.05,0.5], alpha U[0,1] -> rho 0.6, beta~U[0.5,2] per sequence
  c4  M=1000, N=10,000,000, mu~U[0.01,0.05], alpha 1% dense U[0,1] -> rho 0.8,
      beta=1
  c5  M=4096, N=50,000,000, mu~U[0.01,0.05], alpha 0.2% dense -> rho 0.85,
      per-target beta_p~U[0.5,2]
Any of them can be generated at a reduced event count (``n=``) with the same
parameter recipe, which is what the tests do.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "BatchWorkload", "spectral_radius", "rescale_to_radius",
    "simulate_branching", "simulate_thinning_univariate", "make_config",
    "make_batched", "random_params", "cached", "config_params", "c5_params",
]


@dataclass
class Workload:
    """One event sequence plus float32 parameters (the values the GPU sees)."""
    t: np.ndarray            # float64 [n], nondecreasing, t[-1] == T
    m: np.ndarray            # int32 [n], 0 <= m < M
    mu: np.ndarray           # float32 [M]
    alpha: np.ndarray        # float32 [M, M], alpha[target, source]
    beta: np.ndarray         # float32 [1] (shared) or [M] (per target)
    T: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    @property
    def M(self) -> int:
        return int(self.mu.shape[0])

    @property
    def per_target(self) -> bool:
        """True when beta holds one decay per target node."""
        return bool(self.meta.get("per_target", self.beta.shape[0] > 1))


@dataclass
class BatchWorkload:
    """Many independent sequences, concatenated (CSR offsets)."""
    ev_off: np.ndarray       # int64 [S+1]
    m_s: np.ndarray          # int32 [S]
    T_s: np.ndarray          # float64 [S]
    t: np.ndarray            # float64 [sum n]
    m: np.ndarray            # int32 [sum n]
    mu: np.ndarray           # float32, packed: sequence s at sum_{r<s} m_r
    alpha: np.ndarray        # float32, packed: sequence s at sum_{r<s} m_r^2
    beta: np.ndarray         # float32 [S]
    name: str = ""

    @property
    def S(self) -> int:
        return int(self.m_s.shape[0])

    def seq(self, s: int) -> Workload:
        a, b = int(self.ev_off[s]), int(self.ev_off[s + 1])
        M = int(self.m_s[s])
        mo = int(np.sum(self.m_s[:s], dtype=np.int64))
        ao = int(np.sum(self.m_s[:s].astype(np.int64) ** 2))
        return Workload(self.t[a:b], self.m[a:b], self.mu[mo:mo + M],
                        self.alpha[ao:ao + M * M].reshape(M, M), self.beta[s:s + 1],
                        float(self.T_s[s]), name=f"{self.name}[{s}]")


def spectral_radius(a: np.ndarray, tol: float = 1e-12, max_iter: int = 100000) -> float:
    """Spectral radius of a nonnegative matrix (eigvals for small M, else power
    iteration on a damped matrix, which converges for reducible inputs too)."""
    a = np.asarray(a, dtype=np.float64)
    M = a.shape[0]
    if M <= 64:
        return float(np.max(np.abs(np.linalg.eigvals(a))))
    # Perron root of a >= 0: power iteration on a + I (shares eigenvectors,
    # shifts the Perron root by 1 and breaks periodicity).
    b = a + np.eye(M)
    x = np.ones(M) / M
    lam = 0.0
    for _ in range(max_iter):
        y = b @ x
        s = y.sum()
        y /= s
        new = s - 1.0
        if abs(new - lam) <= tol * max(abs(new), 1e-300):
            lam = new
            break
        lam = new
        x = y
    return float(lam)


def rescale_to_radius(a: np.ndarray, rho: float) -> np.ndarray:
    r = spectral_radius(a)
    if r <= 0:
        return a.copy()
    return a * (rho / r)


def random_params(rng: np.random.Generator, M: int, mu_lo: float, mu_hi: float,
                  density: float, rho: float):
    mu = rng.uniform(mu_lo, mu_hi, size=M)
    vals = rng.uniform(0.0, 1.0, size=(M, M))
    if density < 1.0:
        mask = rng.random((M, M)) < density
        vals = np.where(mask, vals, 0.0)
    alpha = rescale_to_radius(vals, rho)
    return mu, alpha


def simulate_branching(rng: np.random.Generator, mu: np.ndarray, alpha: np.ndarray,
                       beta: np.ndarray, T0: float, max_events: int | None = None):
    """Cluster (branching) representation on [0, T0].

    Immigrants of node p: Poisson(mu_p T0) at uniform times.  Each event of
    node q has Poisson(colsum_q) children; a child has node p with probability
    alpha[p, q]/colsum_q and time parent + Exp(rate beta_p) (beta_p is the
    decay of the target's kernel; one shared value if beta has length 1).
    Children after T0 are dropped; generations repeat until none remain.
    Returns (t, m) sorted by time.
    """
    M = mu.shape[0]
    beta = np.broadcast_to(np.asarray(beta, dtype=np.float64), (M,))
    colsum = alpha.sum(axis=0)
    # flat inverse-CDF table over (source q, target p)
    cum = np.cumsum(alpha.T.reshape(-1))          # index q*M + p
    base = np.concatenate(([0.0], np.cumsum(colsum)))[:-1]
    counts = rng.poisson(mu * T0)
    m0 = np.repeat(np.arange(M, dtype=np.int32), counts)
    t0 = rng.uniform(0.0, T0, size=m0.shape[0])
    ts, ms = [t0], [m0]
    pt, pm = t0, m0
    total = t0.shape[0]
    while pt.shape[0] > 0:
        nchild = rng.poisson(colsum[pm])
        if nchild.sum() == 0:
            break
        par_t = np.repeat(pt, nchild)
        par_m = np.repeat(pm, nchild)
        u = rng.random(par_t.shape[0]) * colsum[par_m] + base[par_m]
        idx = np.searchsorted(cum, u, side="right")
        idx = np.minimum(idx, M * M - 1)
        cm = (idx - par_m.astype(np.int64) * M).astype(np.int64)
        # guard against round-off landing on a neighbouring column block
        cm = np.clip(cm, 0, M - 1).astype(np.int32)
        ct = par_t + rng.exponential(1.0, size=par_t.shape[0]) / beta[cm]
        keep = ct <= T0
        pt, pm = ct[keep], cm[keep]
        ts.append(pt)
        ms.append(pm)
        total += pt.shape[0]
        if max_events is not None and total > 50 * max_events:
            raise RuntimeError("branching simulation exploded (supercritical parameters?)")
    t = np.concatenate(ts)
    m = np.concatenate(ms).astype(np.int32)
    order = np.argsort(t, kind="stable")
    return t[order], m[order]


def simulate_thinning_univariate(rng: np.random.Generator, mu: float, alpha: float,
                                 beta: float, n: int):
    """Ogata's thinning for M=1 until n events.  The intensity bound between
    events is the intensity just after the last event (it only decays)."""
    t = np.empty(n)
    s = 0.0          # sum_j exp(-beta (now - t_j)) at time `now`
    now = 0.0
    k = 0
    while k < n:
        lam_bar = mu + alpha * beta * s
        w = rng.exponential(1.0 / lam_bar)
        s *= np.exp(-beta * w)
        now += w
        lam_now = mu + alpha * beta * s
        if rng.random() * lam_bar <= lam_now:
            t[k] = now
            s += 1.0
            k += 1
    return t, np.zeros(n, dtype=np.int32)


def scale_free_digraph(rng: np.random.Generator, M: int, a: float = 0.41, b: float = 0.54,
                       c: float = 0.05, d_in: float = 0.2, d_out: float = 0.0) -> np.ndarray:
    """Directed scale-free graph on M >= 3 nodes, grown by the preferential-
    attachment process of Bollobas, Borgs, Chayes and Riordan (2003) from a
    3-cycle: each step, with probability a a new node v gets an edge v -> w
    (w drawn with probability proportional to its in-degree + d_in); with
    probability b an edge v -> w joins existing nodes (v by out-degree +
    d_out, w by in-degree + d_in); with probability c a new node w gets an
    edge v -> w (v by out-degree + d_out).  Stops once M nodes exist.
    Returns the distinct edges (v, w), v != w, as an int array [E, 2]."""
    if M < 3:
        raise ValueError("the process starts from 3 nodes")
    indeg = np.zeros(M)
    outdeg = np.zeros(M)
    edges = {(0, 1), (1, 2), (2, 0)}
    for v, w in edges:
        outdeg[v] += 1
        indeg[w] += 1
    n = 3

    def pick(deg, delta):
        wgt = deg[:n] + delta
        tot = wgt.sum()
        if tot <= 0.0:
            return int(rng.integers(0, n))
        return int(min(np.searchsorted(np.cumsum(wgt), rng.random() * tot, side="right"), n - 1))

    while n < M:
        r = rng.random()
        if r < a:
            v, w = n, pick(indeg, d_in)
            n += 1
        elif r < a + b:
            v, w = pick(outdeg, d_out), pick(indeg, d_in)
        else:
            v, w = pick(outdeg, d_out), n
            n += 1
        outdeg[v] += 1
        indeg[w] += 1
        if v != w:
            edges.add((v, w))
    return np.array(sorted(edges), dtype=np.int64)


def make_recovery(M: int, n: int, seed: int = 0, mu: float = 0.001, beta: float = 1.0,
                  rho: float = 0.5) -> Workload:
    """Synthetic sequence for the parameter-recovery study: base rate mu for
    every node, one decay beta, alpha on a directed scale-free graph
    (alpha[w, v] > 0 for an edge v -> w: source v excites target w) plus
    self-excitation on the diagonal, weights U[0.5, 1] rescaled to spectral
    radius rho; n events by the cluster representation, T = t_n."""
    rng = np.random.default_rng(np.random.SeedSequence([2604, 1342, 7, M, n, seed]))
    e = scale_free_digraph(rng, M)
    a = np.zeros((M, M))
    a[e[:, 1], e[:, 0]] = rng.uniform(0.5, 1.0, size=e.shape[0])
    a[np.arange(M), np.arange(M)] = rng.uniform(0.5, 1.0, size=M)
    alpha = rescale_to_radius(a, rho)
    mus = np.full(M, mu)
    t, m = _simulate_n(rng, mus, alpha, np.array([beta]), n)
    return Workload(t=t, m=m, mu=mus.astype(np.float32), alpha=alpha.astype(np.float32),
                    beta=np.array([beta], dtype=np.float32), T=float(t[-1]), name=f"recovery_M{M}",
                    meta={"edges": int(e.shape[0]), "rho": rho})


def _expected_rate(mu: np.ndarray, alpha: np.ndarray) -> float:
    M = mu.shape[0]
    return float(np.ones(M) @ np.linalg.solve(np.eye(M) - alpha, mu))


def _simulate_n(rng, mu, alpha, beta, n):
    rate = _expected_rate(mu, alpha)
    T0 = 1.2 * n / rate
    for _ in range(20):
        t, m = simulate_branching(rng, mu, alpha, beta, T0, max_events=n)
        if t.shape[0] >= n:
            return t[:n].copy(), m[:n].copy()
        T0 *= 1.5
    raise RuntimeError("could not simulate enough events")


_FULL_N = {1: 10_000, 2: 1_000_000, 4: 10_000_000, 5: 50_000_000}


def config_params(c: int):
    """(mu, alpha, beta) of single-sequence workload c in {1, 2, 4, 5} as
    float32 (the values the library receives), from seed 1000 c + 1."""
    rp = np.random.Generator(np.random.PCG64(1000 * c + 1))
    if c == 1:
        mu, alpha, beta = np.array([0.5]), np.array([[0.5]]), np.array([1.0])
    elif c == 2:
        mu, alpha = random_params(rp, 16, 0.05, 0.2, 1.0, 0.7)
        beta = np.array([1.0])
    elif c == 4:
        mu, alpha = random_params(rp, 1000, 0.01, 0.05, 0.01, 0.8)
        beta = np.array([1.0])
    elif c == 5:
        mu, alpha = random_params(rp, 4096, 0.01, 0.05, 0.002, 0.85)
        beta = rp.uniform(0.5, 2.0, size=4096)
    else:
        raise ValueError(f"no single-sequence workload {c}")
    return mu.astype(np.float32), alpha.astype(np.float32), beta.astype(np.float32)


def c5_params():
    """Parameters of workload c5 (M = 4096, decay per target node)."""
    return config_params(5)


def make_config(c: int, n: int | None = None) -> Workload:
    """Single-sequence workload c in {1, 2, 4, 5}; ``n`` overrides the event count."""
    if c not in _FULL_N:
        raise ValueError(f"no single-sequence workload {c}")
    N = _FULL_N[c] if n is None else int(n)
    re = np.random.Generator(np.random.PCG64(1000 * c + 2))
    mu32, al32, be32 = config_params(c)
    if c == 1:
        t, m = simulate_thinning_univariate(re, float(mu32[0]), float(al32[0, 0]), float(be32[0]), N)
    if c != 1:
        t, m = _simulate_n(re, mu32.astype(np.float64), al32.astype(np.float64),
                           be32.astype(np.float64), N)
    return Workload(t, m.astype(np.int32), mu32, al32, be32, float(t[-1]),
                    name=f"c{c}", meta={"per_target": c == 5})


def _batched_one(args):
    """One sequence of the batched workload, seeded by its own spawned child."""
    child, lo, hi, M, max_len = args
    rng = np.random.Generator(np.random.PCG64(child))
    L = int(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
    if max_len is not None:
        L = min(L, max_len)
    mu, alpha = random_params(rng, M, 0.05, 0.5, 1.0, 0.6)
    beta = rng.uniform(0.5, 2.0)
    mu32, al32 = mu.astype(np.float32), alpha.astype(np.float32)
    be32 = np.float32(beta)
    t, m = _simulate_n(rng, mu32.astype(np.float64), al32.astype(np.float64),
                       np.array([float(be32)]), L)
    return t, m, mu32, al32.reshape(-1), be32, L


def make_batched(S: int = 4096, lo: int = 100, hi: int = 100_000, M: int = 8,
                 seed: int = 3002, max_len: int | None = None,
                 workers: int | None = None) -> BatchWorkload:
    """Workload c3: S independent sequences with their own parameters.
    ``max_len`` caps every length (for quick tests) without changing seeds.
    Sequences are simulated in ``workers`` processes (default: up to 16 host
    cores); each is seeded by its own child of SeedSequence(seed), so the
    result does not depend on the worker count."""
    children = np.random.SeedSequence(seed).spawn(S)
    jobs = [(children[s], lo, hi, M, max_len) for s in range(S)]
    if workers is None:
        workers = int(os.environ.get("HAWKES_GEN_WORKERS", min(16, os.cpu_count() or 1)))
    if workers > 1 and S >= 64:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_batched_one, jobs, chunksize=max(1, S // (8 * workers)))
    else:
        res = [_batched_one(j) for j in jobs]
    ts, ms, mus, als, bes, lens = zip(*res)
    Ts = [float(t[-1]) for t in ts]
    ev_off = np.zeros(S + 1, dtype=np.int64)
    ev_off[1:] = np.cumsum(lens)
    return BatchWorkload(ev_off, np.full(S, M, dtype=np.int32), np.array(Ts),
                         np.concatenate(ts), np.concatenate(ms).astype(np.int32),
                         np.concatenate(mus), np.concatenate(als),
                         np.array(bes, dtype=np.float32), name="c3")


def cached(key: str, fn):
    """Memoise a workload on disk (npz, no pickles) under $HAWKES_CACHE_DIR
    (default /tmp/hawkes_workloads)."""
    d = os.environ.get("HAWKES_CACHE_DIR", "/tmp/hawkes_workloads")
    os.makedirs(d, exist_ok=True)
    path = os.path.join(d, key + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        if "ev_off" in z:
            return BatchWorkload(z["ev_off"], z["m_s"], z["T_s"], z["t"], z["m"], z["mu"],
                                 z["alpha"], z["beta"], name=str(z["name"]))
        return Workload(z["t"], z["m"], z["mu"], z["alpha"], z["beta"], float(z["T"]),
                        name=str(z["name"]), meta={"per_target": bool(z["per_target"])})
    w = fn()
    tmp = path + f".tmp{os.getpid()}.npz"
    if isinstance(w, BatchWorkload):
        np.savez(tmp, ev_off=w.ev_off, m_s=w.m_s, T_s=w.T_s, t=w.t, m=w.m, mu=w.mu,
                 alpha=w.alpha, beta=w.beta, name=w.name)
    else:
        np.savez(tmp, t=w.t, m=w.m, mu=w.mu, alpha=w.alpha, beta=w.beta, T=w.T, name=w.name,
                 per_target=w.meta.get("per_target", False))
    os.replace(tmp, path)
    return w
