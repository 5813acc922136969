"""Full-size parity: every workload at its published size, in the same launch
configuration the benchmark times, against the FP64 oracle.

Gradients are gated at the perturbed point theta_pert = (1.25 mu, 0.8 alpha,
1.2 beta): at the generating parameters the gradient is a near-cancelling
difference of O(N) terms (the statistical noise of the fit), so a plain
relative error there measures cancellation rather than the kernels.  The
log-likelihood is gated at both points.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import rel_err, scalar_rel

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01342_amd as H
    H.lib()
    return H


def _gpu(H, w, mu, al, be, chunk_log2=0):
    import torch
    d = "cuda"
    g = H.loglik_grad(torch.as_tensor(w.t, device=d), torch.as_tensor(w.m, device=d),
                      torch.as_tensor(mu, device=d), torch.as_tensor(al, device=d), torch.as_tensor(be, device=d),
                      w.T, chunk_log2)
    torch.cuda.synchronize()
    return g[0].item(), g[1].cpu().numpy(), g[2].cpu().numpy(), g[3].cpu().numpy()


def _pert(w):
    return ((1.25 * w.mu).astype(np.float32), (0.8 * w.alpha).astype(np.float32),
            (1.2 * w.beta).astype(np.float32))


def _report(label, g, r):
    e = (scalar_rel(g[0], r[0]), rel_err(g[1], r[1]), rel_err(g[2], np.reshape(r[2], g[2].shape)),
         rel_err(g[3], np.ravel(r[3])))
    print(f"{label}: loglik {e[0]:.2e} mu {e[1]:.2e} alpha {e[2]:.2e} beta {e[3]:.2e}", flush=True)
    return e


@pytest.mark.timeout(300)
def test_c2_full(H):
    from paper_2604_01342_amd import workloads as W
    w = W.cached("c2_full", lambda: W.make_config(2))
    assert w.n == 1_000_000 and w.M == 16
    r = oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T)
    e = _report("c2 theta_true", _gpu(H, w, w.mu, w.alpha, w.beta), r)
    assert e[0] < TOL
    mu, al, be = _pert(w)
    e = _report("c2 theta_pert", _gpu(H, w, mu, al, be), oracle.forward(w.t, w.m, mu, al, be, w.T))
    assert max(e) < TOL


@pytest.mark.timeout(300)
def test_c4_full(H):
    from paper_2604_01342_amd import workloads as W
    w = W.cached("c4_full", lambda: W.make_config(4))
    assert w.n == 10_000_000 and w.M == 1000
    mu, al, be = _pert(w)
    g = _gpu(H, w, mu, al, be, 20)
    print("c4 gpu done; running the FP64 oracle over 1e7 events (about 40 s)", flush=True)
    e = _report("c4 theta_pert (chunks of 2^20)", g, oracle.forward(w.t, w.m, mu, al, be, w.T))
    assert max(e) < TOL


@pytest.mark.timeout(600)
def test_c3_full(H):
    """All 4096 sequences in one batched launch; the oracle checks a fixed
    sample of them (every 32nd, plus the shortest and the longest)."""
    import torch
    from paper_2604_01342_amd import workloads as W
    bw = W.cached("c3_full", lambda: W.make_batched())
    assert bw.S == 4096
    b = H.Batch.from_numpy(bw)
    ll, gmu, ga, gb = [x.cpu().numpy() for x in H.loglik_grad_batched(b)]
    torch.cuda.synchronize()
    lens = np.diff(bw.ev_off)
    sample = sorted(set(range(0, bw.S, 32)) | {int(np.argmin(lens)), int(np.argmax(lens))})
    mo = np.concatenate([[0], np.cumsum(bw.m_s.astype(np.int64))])
    ao = np.concatenate([[0], np.cumsum(bw.m_s.astype(np.int64) ** 2)])
    worst = np.zeros(4)
    for s in sample:
        w = bw.seq(s)
        r = oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T)
        worst[0] = max(worst[0], scalar_rel(ll[s], r[0]))
        worst[1] = max(worst[1], rel_err(gmu[mo[s]:mo[s + 1]], r[1]))
        worst[2] = max(worst[2], rel_err(ga[ao[s]:ao[s + 1]], np.ravel(r[2])))
        worst[3] = max(worst[3], rel_err(gb[s:s + 1], r[3]))
    print(f"c3 4096 sequences, {bw.ev_off[-1]} events, oracle on {len(sample)} sampled: worst errors "
          f"loglik {worst[0]:.2e} mu {worst[1]:.2e} alpha {worst[2]:.2e} beta {worst[3]:.2e}", flush=True)
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(gb))
    # dL/dbeta of a short sequence at its generating point can be a near-zero
    # difference; the small-M engine keeps float64 state, so it still matches
    assert max(worst) < TOL


@pytest.mark.timeout(300)
def test_c5_prefix_1e6(H):
    """c5 (M = 4096, per-target decays) on its first 1e6 events, against
    oracle results stored by tests/golden/make_c5_prefix.py (the O(N M)
    per-target oracle takes minutes there).  dL/dalpha is compared on the
    stored sample of 20,000 entries: the normwise error is estimated from the
    sample's squared errors scaled to all M^2 entries."""
    import hashlib
    import os
    from paper_2604_01342_amd import workloads as W
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "c5_prefix_1e6.npz"), allow_pickle=False)
    n = int(gold["n"])
    w = W.cached("c5_1e6", lambda: W.make_config(5, n=n))
    h = hashlib.sha256()
    for a in (w.t, w.m, w.mu, w.alpha, w.beta, np.float64(w.T)):
        h.update(np.ascontiguousarray(a).tobytes())
    assert h.hexdigest() == str(gold["sha256"]), "regenerated c5 inputs differ from the stored oracle's"
    lt = _gpu(H, w, w.mu, w.alpha, w.beta, 20)[0]
    mu, al, be = _pert(w)
    lp, gmu, ga, gb = _gpu(H, w, mu, al, be, 20)
    idx = gold["ga_idx"]
    d = np.ravel(ga)[idx] - gold["ga_val"]
    ga_est = float(np.sqrt(np.sum(d * d) * (w.M * w.M / idx.size)) / float(gold["ga_norm"]))
    e = (scalar_rel(lt, float(gold["loglik_true"])), scalar_rel(lp, float(gold["loglik_pert"])),
         rel_err(gmu, gold["g_mu"]), ga_est, rel_err(gb, gold["g_beta"]))
    print(f"c5 first 1e6 events: loglik theta_true {e[0]:.2e}; theta_pert loglik {e[1]:.2e} mu {e[2]:.2e} "
          f"alpha {e[3]:.2e} (sampled estimate) beta {e[4]:.2e}", flush=True)
    assert max(e) < TOL
