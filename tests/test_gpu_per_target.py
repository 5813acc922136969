"""GPU parity for one decay per target node (beta[M]): the HIP library's
per-target path against the FP64 oracle's reverse-mode pass and, on tiny
inputs, the O(N^2) definition.  Same tolerance as the shared-decay path:
1e-6 relative on the log-likelihood and normwise on each gradient block."""
import numpy as np
import pytest

import oracle
from tests.helpers import rand_problem, rel_err, scalar_rel
from tests.test_gpu_parity import H, check, run_gpu  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.mark.timeout(300)
@pytest.mark.parametrize("seed,n,M,density,ties,chunk", [
    (31, 1, 3, 1.0, False, 0), (32, 60, 2, 1.0, True, 0), (33, 500, 9, 1.0, False, 0),
    (34, 3000, 33, 0.3, False, 0), (35, 9000, 70, 0.1, True, 12), (36, 20000, 130, 0.05, False, 12),
    (37, 4097, 64, 1.0, False, 12), (38, 5000, 5, 1.0, True, 0), (39, 12000, 200, 0.02, False, 12)])
def test_per_target_matches_adjoint_oracle(H, seed, n, M, density, ties, chunk):
    t, m, mu, alpha, beta, T = rand_problem(seed, n, M, per_target=True, ties=ties, density=density, rate=20.0)
    assert beta.shape == (M,)
    ref = oracle.adjoint(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, chunk), ref, label=f"per-target n={n} M={M} chunk={chunk}")


# The dense adjoint kernel handles a window of records by one of three forms,
# chosen by its largest decay exponent beta_max (t_first - t_last): short
# (<= 0.5), merged (up to 64) and pairwise-exact (beyond).  Stretches of
# 5000, 20 and 0.1 events per unit time, with beta_p in [0.5, 2] and windows
# of about 64 records per node block, give every form and every change
# between two forms; M = 150 (three node blocks) adds blocks whose two record
# lists differ.
@pytest.mark.timeout(300)
@pytest.mark.parametrize("M,chunk", [(20, 0), (150, 12)])
def test_per_target_window_forms(H, M, chunk):
    rng = np.random.default_rng(90 + M)
    parts = [(3000, 5000.0), (3000, 20.0), (400, 0.1), (3000, 5000.0), (2000, 20.0), (300, 0.1)]
    t = np.cumsum(np.concatenate([rng.exponential(1.0 / r, size=k) for k, r in parts]))
    n = t.size
    m = rng.integers(0, M, size=n).astype(np.int32)
    mu = rng.uniform(0.05, 0.5, size=M).astype(np.float32)
    a = rng.uniform(0.0, 1.0, size=(M, M)) * (rng.random((M, M)) < 0.3)
    alpha = (a * (0.5 / a.sum(axis=0).max())).astype(np.float32)
    beta = rng.uniform(0.5, 2.0, size=M).astype(np.float32)
    T = float(t[-1] + 0.5)
    # the stretches' spans over 64 events of one node block, times beta_max
    blocks = (M + 63) // 64
    spans = [float(beta.max()) * 64 * blocks / r for _, r in parts]
    assert min(spans) < 0.5 and any(0.5 < x < 64 for x in spans) and max(spans) > 64
    ref = oracle.adjoint(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, chunk), ref, label=f"per-target window forms M={M} chunk={chunk}")


# Columns of alpha longer than the forward kernel's stage (1136 entries) and
# the segment aggregation's (2048): every event's column is pushed straight
# from global memory, a whole column per pass group.
@pytest.mark.timeout(300)
def test_per_target_columns_past_the_stages(H):
    t, m, mu, alpha, beta, T = rand_problem(57, 2500, 2100, per_target=True, density=1.0, rate=40.0)
    ref = oracle.adjoint(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, 0), ref, label="per-target M=2100 dense columns")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,M", [(64 * 4096, 20), (64 * 4096 + 1, 20), (300_000, 30), (4096 * 200 + 77, 12)])
def test_per_target_gradient_checkpoint_levels(H, n, M):
    # the gradient keeps chunk-start states in 64 level-1 slots: 64 chunks of
    # 2^12 events take one level, one event more makes two chunks per slot
    # (level-2 slots refilled per block in the reverse sweep), and so on
    t, m, mu, alpha, beta, T = rand_problem(60 + M, n, M, per_target=True, density=0.3, rate=20.0)
    ref = oracle.adjoint(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, 12), ref, label=f"per-target checkpoints n={n} M={M} chunk=12")


def test_per_target_node_limit(H):
    # the per-target forward kernel keeps 32 bytes of LDS per node plus 24 KiB
    # of staging and batch tables: M <= 4352 under MI355X's 160 KiB per workgroup,
    # one node more is refused on the host before any launch
    import torch
    from tests.test_gpu_parity import dev
    for M, ok in ((4352, True), (4353, False)):
        t, m, mu, alpha, beta, T = rand_problem(73, 3000, M, per_target=True, density=0.001, rate=20.0)
        args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                dev(beta, torch.float32), T)
        if ok:
            L = H.loglik(*args).item()
            assert scalar_rel(L, oracle.adjoint(t, m, mu, alpha, beta, T, grad=False)) < TOL
        else:
            with pytest.raises(H.HawkesError) as e:
                H.loglik(*args)
            assert e.value.status == 4


def test_per_target_matches_definition_tiny(H):
    t, m, mu, alpha, beta, T = rand_problem(41, 120, 4, per_target=True, ties=True, rate=3.0)
    ref = oracle.brute(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T), ref, label="per-target vs definition")


def test_per_target_reduces_to_shared_decay(H):
    """beta_p all equal: the per-target path must give the shared-decay answer
    (dL/dbeta summed over targets is the shared-decay derivative)."""
    t, m, mu, alpha, beta1, T = rand_problem(42, 8000, 40, density=0.3, rate=20.0)
    beta_m = np.full(40, beta1[0], np.float32)
    g_pt = run_gpu(H, t, m, mu, alpha, beta_m, T, 12)
    ref = oracle.forward(t, m, mu, alpha, beta1, T)
    errs = (scalar_rel(g_pt[0], ref[0]), rel_err(g_pt[1], ref[1]), rel_err(g_pt[2], ref[2][0]),
            scalar_rel(float(np.sum(g_pt[3])), float(ref[3][0])))
    print("per-target with equal decays vs shared-decay oracle:", errs, flush=True)
    assert max(errs) < TOL


def test_per_target_chunk_invariance_and_determinism(H):
    t, m, mu, alpha, beta, T = rand_problem(43, 30000, 50, per_target=True, density=0.2, rate=30.0)
    a = run_gpu(H, t, m, mu, alpha, beta, T, 12)
    b = run_gpu(H, t, m, mu, alpha, beta, T, 20)
    c = run_gpu(H, t, m, mu, alpha, beta, T, 12)
    assert scalar_rel(a[0], b[0]) < 1e-9
    for x, y in zip(a[1:], b[1:]):
        assert rel_err(x, y) < 1e-7
    # repeatable bitwise except dL/dalpha (several waves add into one LDS
    # tile in a varying order): to rounding there
    assert a[0] == c[0]
    assert np.array_equal(a[1], c[1]) and np.array_equal(a[3], c[3])
    assert rel_err(a[2], c[2]) < 1e-13


def test_per_target_loglik_only_and_intensity(H):
    import torch
    from tests.test_gpu_parity import dev
    t, m, mu, alpha, beta, T = rand_problem(44, 6000, 30, per_target=True, density=0.3, rate=20.0)
    L = H.loglik(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                 dev(beta, torch.float32), T, 12)
    torch.cuda.synchronize()
    assert scalar_rel(float(L.item()), oracle.adjoint(t, m, mu, alpha, beta, T, grad=False)) < TOL
    lam = H.intensity(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                      dev(alpha, torch.float32), dev(beta, torch.float32), T, 12).cpu().numpy()
    idx = np.arange(0, len(t), 7)
    ref = oracle.intensity_at(t, m, mu, alpha, beta, idx)
    assert np.max(np.abs(lam[idx] - ref) / ref) < 2e-6


def test_per_target_empty(H):
    M = 12
    t = np.zeros(0); m = np.zeros(0, np.int32)
    mu = np.full(M, 0.3, np.float32); alpha = np.full((M, M), 0.01, np.float32)
    beta = np.linspace(0.5, 2.0, M).astype(np.float32)
    L, gmu, ga, gb = run_gpu(H, t, m, mu, alpha, beta, 2.0)
    assert L == pytest.approx(-2.0 * float(mu.astype(np.float64).sum()), rel=1e-12)
    np.testing.assert_allclose(gmu, -2.0)
    np.testing.assert_allclose(ga, 0.0)
    np.testing.assert_allclose(gb, 0.0)


@pytest.mark.timeout(300)
def test_c5_reduced(H):
    """The M = 4096, 0.2%-dense, per-target-decay workload, generated at 2e4
    events (the O(N M) oracle takes about 5 s per pass there)."""
    from paper_2604_01342_amd import workloads as W
    w = W.cached("c5_20k", lambda: W.make_config(5, n=20_000))
    assert w.M == 4096 and w.beta.shape == (4096,)
    ref = oracle.adjoint(w.t, w.m, w.mu, w.alpha, w.beta, w.T)
    check(run_gpu(H, w.t, w.m, w.mu, w.alpha, w.beta, w.T, 16), ref, label="c5 first 2e4 events")
    mu = (1.25 * w.mu).astype(np.float32)
    al = (0.8 * w.alpha).astype(np.float32)
    be = (1.2 * w.beta).astype(np.float32)
    check(run_gpu(H, w.t, w.m, mu, al, be, w.T, 16), oracle.adjoint(w.t, w.m, mu, al, be, w.T),
          label="c5 first 2e4 events, theta_pert")
