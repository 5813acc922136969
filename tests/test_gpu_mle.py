"""The fused maximum-likelihood step (hawkes_adam_step through the AdamMLE
binding): Adam arithmetic against a NumPy restatement driven by the FP64
oracle's gradients, and HIP-graph replays against eager steps."""
import numpy as np
import pytest

import oracle
from tests.helpers import rand_problem
from tests.test_gpu_parity import H  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _adam_reference(t, m, mu, al, be, T, steps, lr=0.05, b1=0.9, b2=0.999, eps=1e-8, floor=1e-6,
                    per_target=False, lam=0.0, h=0.05, log_mu=False, log_beta=False, log_alpha=False):
    """Projected Adam on -L/n plus the oracle's hinge-l1 penalty (weight lam,
    hinge h, decided in float32), with the oracle's gradient; moments and
    parameters rounded to float32 after each update, as the library stores
    them.  log_mu / log_beta: the step acts on log x (gradient times x,
    x <- x exp(-step))."""
    n = max(len(t), 1)
    x = [mu.astype(np.float32).copy(), al.astype(np.float32).copy(), be.astype(np.float32).copy()]
    lo = [floor, 0.0, floor]
    mom = [np.zeros_like(v) for v in x]
    vel = [np.zeros_like(v) for v in x]
    traj = []
    for k in range(1, steps + 1):
        f = oracle.adjoint if per_target else oracle.forward
        L, gmu, ga, gb = f(t, m, x[0], x[1], x[2], T)
        grads = [np.asarray(gmu), np.reshape(ga, x[1].shape), np.reshape(gb, x[2].shape)]
        c1, c2 = 1.0 - b1 ** k, 1.0 - b2 ** k
        pen = oracle.sparsity_penalty(x[1], lam, np.float32(h))[1]
        for j in range(3):
            g = -grads[j] / n + (pen if j == 1 else 0.0)
            lg = (j == 0 and log_mu) or (j == 2 and log_beta) or (j == 1 and log_alpha)
            if lg:
                g = g * x[j].astype(np.float64)
            mn = b1 * mom[j].astype(np.float64) + (1 - b1) * g
            vn = b2 * vel[j].astype(np.float64) + (1 - b2) * g * g
            mom[j] = mn.astype(np.float32)
            vel[j] = vn.astype(np.float32)
            stp = lr * (mn / c1) / (np.sqrt(vn / c2) + eps)
            xn = x[j].astype(np.float64) * np.exp(-stp) if lg else x[j].astype(np.float64) - stp
            x[j] = np.maximum(xn, lo[j]).astype(np.float32)
        traj.append((L, [v.copy() for v in x]))
    return traj


# lam > 0: the penalised objective; the hinge 0.07 is no multiple of the
# learning rate, so that no entry lands on it exactly (an entry one float32
# ulp either side of h would take different branches on the two sides)
@pytest.mark.parametrize("per_target,M,lam,logs", [(False, 3, 0.0, False), (False, 40, 0.0, False),
                                                   (True, 20, 0.0, False), (False, 3, 0.1, False),
                                                   (False, 40, 0.1, False), (True, 20, 0.1, False),
                                                   (False, 3, 0.1, True), (False, 40, 0.1, True),
                                                   (True, 20, 0.0, True), (False, 40, 0.1, "all"),
                                                   (True, 20, 0.1, "all")])
def test_adam_steps_match_reference(H, per_target, M, lam, logs):
    import torch
    t, m, mu, al, be, T = rand_problem(51 + M, 3000, M, per_target=per_target, density=0.5, rate=10.0)
    ref = _adam_reference(t, m, mu, al, be, T, 4, per_target=per_target, lam=lam, h=0.07, log_mu=bool(logs),
                          log_beta=bool(logs), log_alpha=logs == "all")
    d = "cuda"
    opt = H.AdamMLE(torch.as_tensor(t, device=d), torch.as_tensor(m, device=d), torch.as_tensor(mu, device=d),
                    torch.as_tensor(al, device=d), torch.as_tensor(be, device=d), T, lambda1=lam, h=0.07,
                    log_mu=bool(logs), log_beta=bool(logs), log_alpha=logs == "all")
    for k, (Lr, xr) in enumerate(ref):
        L = float(opt.step().item())
        torch.cuda.synchronize()
        assert abs(L - Lr) <= 1e-6 * abs(Lr), (k, L, Lr)
        got = [opt.mu.cpu().numpy(), opt.alpha.cpu().numpy(), opt.beta.cpu().numpy()]
        for g, r in zip(got, xr):
            np.testing.assert_allclose(g, r, rtol=2e-6, atol=1e-7)


@pytest.mark.parametrize("per_target", [False, True])
def test_graph_replays_equal_eager_steps(H, per_target):
    """A captured step, replayed several times with eager work and
    synchronisations in between, must give bitwise the parameters and
    log-likelihoods of the same number of eager steps."""
    import torch
    t, m, mu, al, be, T = rand_problem(61, 20000, 70, per_target=per_target, density=0.1, rate=20.0)
    d = "cuda"
    args = [torch.as_tensor(x, device=d) for x in (t, m, mu, al, be)]
    eager = H.AdamMLE(*args, T, chunk_log2=12)
    graph = H.AdamMLE(*args, T, chunk_log2=12)
    Le = [float(eager.step().item())]
    Lg = [float(graph.step().item())]
    torch.cuda.synchronize()
    graph.capture()
    for k in range(4):
        Le.append(float(eager.step().item()))
        _ = torch.ones(1000, device=d).sum()   # unrelated eager work between replays
        Lg.append(float(graph.replay().item()))
        torch.cuda.synchronize()
        assert Le[-1] == Lg[-1], (k, Le[-1], Lg[-1])
        for a, b in ((eager.mu, graph.mu), (eager.alpha, graph.alpha), (eager.beta, graph.beta)):
            assert torch.equal(a, b)


def test_parameter_recovery_small(H):
    """The training loop end to end, at a small size of the paper's recovery
    study: a sequence simulated from known parameters (alpha on a directed
    scale-free graph plus self-excitation, mu = 0.001, beta = 1), fitted by
    500 graph-replayed Adam steps on the penalised per-event NLL (lr 0.05,
    lambda1 0.1, h 0.05, steps on log mu and log beta) from a fixed start.
    Measured: relative l2 errors 1.7% (mu), 3.4% (alpha), 0.3% (beta); the
    bounds leave about 3x room.  The fit must be at least as likely as the
    generating parameters (to 1e-4 per event: the penalty pulls it away from
    the unpenalised maximum)."""
    import torch
    from paper_2604_01342_amd import workloads as W
    M, n = 10, 100_000
    w = W.make_recovery(M, n)
    d = "cuda"
    t = torch.as_tensor(w.t, device=d)
    m = torch.as_tensor(w.m, device=d)
    opt = H.AdamMLE(t, m, torch.full((M,), n / (M * w.T), dtype=torch.float32, device=d),
                    torch.full((M, M), 0.1 / M, dtype=torch.float32, device=d),
                    torch.full((1,), 0.5, dtype=torch.float32, device=d), w.T, lr=0.05, lambda1=0.1, h=0.05,
                    log_mu=True, log_beta=True)
    opt.step()
    torch.cuda.synchronize()
    opt.capture()
    for _ in range(499):
        opt.replay()
    torch.cuda.synchronize()

    def rel(a, b):
        a = np.asarray(a, dtype=np.float64).ravel()
        b = np.asarray(b, dtype=np.float64).ravel()
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    e_mu = rel(opt.mu.cpu().numpy(), w.mu)
    e_al = rel(opt.alpha.cpu().numpy(), w.alpha)
    e_be = rel(opt.beta.cpu().numpy(), w.beta)
    L_fit = float(H.loglik(t, m, opt.mu, opt.alpha, opt.beta, w.T).item()) / n
    L_true = float(oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T, grad=False)) / n
    print(f"recovery M={M} n={n}: errors mu {e_mu:.3e} alpha {e_al:.3e} beta {e_be:.3e}; "
          f"L/n fit {L_fit:.6f} truth {L_true:.6f}", flush=True)
    assert e_mu < 0.05 and e_al < 0.1 and e_be < 0.01
    assert L_fit > L_true - 1e-4
