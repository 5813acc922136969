"""Stored FP64 oracle results for the first 1e6 events of the c5 workload
(M = 4096, alpha 0.2% dense, spectral radius 0.85, one decay per target node
drawn from U[0.5, 2]).

The per-target oracle costs O(N M) per pass, about seven minutes here for
1e6 events, too long for a test, so this script runs it once and stores what
the GPU test compares against.  It calls only the oracle (oracle/) and the
seeded workload generator; nothing here touches the HIP library.

Stored (c5_prefix_1e6.npz):
  sha256       of the generated inputs (times, marks, mu, alpha, beta, T),
               so that the test can check that it regenerated the same ones
  loglik_true  log-likelihood at the generating parameters
  loglik_pert  log-likelihood at theta_pert = (1.25 mu, 0.8 alpha, 1.2 beta)
  g_mu, g_beta the full gradient blocks at theta_pert
  ga_idx, ga_val  20,000 entries of dL/dalpha at theta_pert (flat indices
               drawn without replacement from a fixed seed), ga_norm its
               Frobenius norm

Run from the repository root: python tests/golden/make_c5_prefix.py
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2604_01342_amd import workloads as W  # noqa: E402

N = 1_000_000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_prefix_1e6.npz")


def inputs_sha256(w) -> str:
    h = hashlib.sha256()
    for a in (w.t, w.m, w.mu, w.alpha, w.beta, np.float64(w.T)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def pert(w):
    return ((1.25 * w.mu).astype(np.float32), (0.8 * w.alpha).astype(np.float32),
            (1.2 * w.beta).astype(np.float32))


def main():
    t0 = time.time()
    w = W.make_config(5, n=N)
    print(f"generated n={w.n} M={w.M} T={w.T:.3f} ({time.time() - t0:.1f}s)", flush=True)
    sha = inputs_sha256(w)
    t0 = time.time()
    lt = oracle.adjoint(w.t, w.m, w.mu, w.alpha, w.beta, w.T, grad=False)
    print(f"theta_true loglik {lt!r} ({time.time() - t0:.1f}s)", flush=True)
    mu, al, be = pert(w)
    t0 = time.time()
    lp, gmu, ga, gb = oracle.adjoint(w.t, w.m, mu, al, be, w.T)
    print(f"theta_pert loglik {lp!r} ({time.time() - t0:.1f}s)", flush=True)
    rng = np.random.Generator(np.random.PCG64(2604))
    idx = np.sort(rng.choice(w.M * w.M, size=20_000, replace=False)).astype(np.int64)
    np.savez_compressed(OUT, sha256=np.array(sha), n=np.int64(N), loglik_true=np.float64(lt),
                        loglik_pert=np.float64(lp), g_mu=gmu, g_beta=gb, ga_idx=idx,
                        ga_val=ga.ravel()[idx], ga_norm=np.float64(np.linalg.norm(ga)))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
