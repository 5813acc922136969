"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances follow the precision plan: float32 decays, state and intensities,
float64 time differences and float64 sums, so the log-likelihood and each
gradient block must match the oracle to 1e-6 relative (normwise for vectors
and matrices).
"""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import rand_problem, rel_err, scalar_rel

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


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def run_gpu(H, t, m, mu, alpha, beta, T, chunk_log2=0):
    import torch
    L, gmu, ga, gb = H.loglik_grad(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                                   dev(alpha, torch.float32), dev(beta, torch.float32), T, chunk_log2)
    torch.cuda.synchronize()
    return float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()


def check(gpu, ref, tol=TOL, label=""):
    L, gmu, ga, gb = gpu
    Lr, gmur, gar, gbr = ref
    errs = (scalar_rel(L, Lr), rel_err(gmu, gmur), rel_err(ga, np.reshape(gar, np.shape(ga))),
            rel_err(gb, np.ravel(gbr)))
    print(f"{label} errors: L {errs[0]:.2e} mu {errs[1]:.2e} alpha {errs[2]:.2e} beta {errs[3]:.2e}", flush=True)
    assert errs[0] <= tol, f"loglik rel err {errs[0]}"
    assert errs[1] <= tol, f"g_mu rel err {errs[1]}"
    assert errs[2] <= tol, f"g_alpha rel err {errs[2]}"
    assert errs[3] <= tol, f"g_beta rel err {errs[3]}"
    return errs


# ------------------------------------------------------------- small engine (M <= 8)
@pytest.mark.parametrize("seed,n,M,ties", [(1, 1, 1, False), (2, 2, 1, False), (3, 100, 2, True),
                                           (4, 3000, 3, False), (5, 5000, 5, True), (6, 20000, 8, False),
                                           (7, 777, 7, True), (8, 70000, 4, False)])
def test_small_engine_matches_oracle(H, seed, n, M, ties):
    t, m, mu, alpha, beta, T = rand_problem(seed, n, M, ties=ties, rate=2.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T), ref, label=f"small n={n} M={M}")


def test_empty_sequence(H):
    for M in (3, 20):
        t = np.zeros(0); m = np.zeros(0, np.int32)
        mu = np.full(M, 0.3, np.float32); alpha = np.full((M, M), 0.01, np.float32); beta = np.ones(1, np.float32)
        L, gmu, ga, gb = run_gpu(H, t, m, mu, alpha, beta, 2.0)
        assert L == pytest.approx(-2.0 * float(mu.astype(np.float64).sum()), rel=1e-12)
        np.testing.assert_allclose(gmu, -2.0)
        np.testing.assert_allclose(ga, 0.0)
        np.testing.assert_allclose(gb, 0.0)


# ------------------------------------------------------------- large engine (M > 8)
@pytest.mark.parametrize("seed,n,M,density,ties,chunk", [(11, 1, 9, 1.0, False, 0), (12, 500, 16, 1.0, True, 0),
                                                         (13, 5000, 33, 0.3, False, 0),
                                                         (14, 9000, 70, 0.1, True, 12),
                                                         (15, 20000, 130, 0.05, False, 12),
                                                         (16, 4097, 64, 1.0, False, 12)])
def test_large_engine_matches_oracle(H, seed, n, M, density, ties, chunk):
    t, m, mu, alpha, beta, T = rand_problem(seed, n, M, ties=ties, density=density, rate=20.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, chunk), ref, label=f"large n={n} M={M} chunk={chunk}")


# ------------------------------------------------------------- support-restricted dL/dalpha
# hawkes_loglik_grad_support: the oracle's dense gradient with the entries off
# alpha's support set to zero.  Large engine: rows with more nonzeros than the
# forward pass keeps in registers (16), several chunks, anchored records
# (rate 20) and per-record decays (rate 1: segments spanning beta u > 600),
# M = 2600 (node records above 64 KiB of LDS); small engine and per-target decays: the dense gradient, masked.
@pytest.mark.parametrize("seed,n,M,density,per_target,chunk,rate",
                         [(81, 6000, 4, 0.5, False, 0, 2.0), (82, 30000, 120, 0.3, False, 12, 20.0),
                          (83, 20000, 300, 0.01, False, 0, 20.0), (84, 12000, 40, 0.5, False, 12, 1.0),
                          (85, 4000, 24, 0.3, True, 12, 5.0), (86, 1, 9, 1.0, False, 0, 1.0),
                          (87, 12000, 2600, 0.002, False, 0, 20.0)])
def test_support_gradient_is_the_masked_dense_gradient(H, seed, n, M, density, per_target, chunk, rate):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(seed, n, M, per_target=per_target, density=density, rate=rate)
    Lr, gmur, gar, gbr = (oracle.adjoint if per_target else oracle.forward)(t, m, mu, alpha, beta, T)
    gar = np.where(alpha != 0.0, np.reshape(gar, (M, M)), 0.0)
    L, gmu, ga, gb = H.loglik_grad(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                                   dev(alpha, torch.float32), dev(beta, torch.float32), T, chunk, support=True)
    torch.cuda.synchronize()
    got = (float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy())
    check(got, (Lr, gmur, gar, gbr), label=f"support n={n} M={M} pt={per_target} chunk={chunk}")
    assert np.all(got[2][alpha == 0.0] == 0.0)
    assert int(np.count_nonzero(alpha)) > 0


@pytest.mark.parametrize("cols,ranges,chunk,rows", [(64, 0, 0, 0), (64, 2, 12, 0), (128, 0, 0, 0), (128, 2, 12, 0),
                                                   (0, 1, 0, 0), (0, 2, 12, 0), (0, 64, 0, 0), (0, 1024, 0, 0),
                                                   (256, 0, 0, 0), (256, 8, 12, 0), (256, 0, 0, 32),
                                                   (256, 1, 12, 32), (256, 64, 0, 32), (256, 16, 14, 16)])
def test_dense_layouts_match_oracle(H, cols, ranges, chunk, rows):
    # the dense dL/dalpha kernel's tile width (64, 128 or 256 nodes, set
    # through the launch tuning), height (16 rows with float64 register
    # accumulators, 32 with float32 ones flushed into a float64 tile) and
    # event-range count change its run, slot and workgroup layout, never the
    # result beyond rounding
    t, m, mu, alpha, beta, T = rand_problem(17, 30000, 200, density=0.1, rate=40.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    try:
        H.set_tuning(dense_cols=cols, dense_ranges=ranges, dense_rows=rows)
        got = run_gpu(H, t, m, mu, alpha, beta, T, chunk)
    finally:
        H.set_tuning()
    check(got, ref, label=f"dense layout cols={cols or 'auto'} ranges={ranges or 'auto'} chunk={chunk} "
                          f"rows={rows or 'auto'}")


@pytest.mark.parametrize("M,rows", [(400, 0), (1000, 16), (777, 32)])
def test_dense_row_heights_at_large_m(H, M, rows):
    # 32-row float32-accumulator tiles are the rule from 384 nodes; both
    # heights against the oracle at several chunks, with rows past M
    t, m, mu, alpha, beta, T = rand_problem(18 + M, 60000, M, density=0.02, rate=60.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    try:
        H.set_tuning(dense_rows=rows)
        got = run_gpu(H, t, m, mu, alpha, beta, T, 14)
    finally:
        H.set_tuning()
    check(got, ref, label=f"dense rows={rows or 'auto'} M={M}")


@pytest.mark.parametrize("item_log2", [4, 6, 9, 12])
def test_small_item_lengths_match_oracle(H, item_log2):
    # the small-M engine's events per lane item (launch tuning) change its
    # item, tile and reduction layout, never the result
    t, m, mu, alpha, beta, T = rand_problem(5, 20000, 6, ties=True, rate=3.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    try:
        H.set_tuning(item_log2=item_log2)
        got = run_gpu(H, t, m, mu, alpha, beta, T)
    finally:
        H.set_tuning()
    check(got, ref, label=f"small item_log2={item_log2}")


def test_chunk_size_invariance(H):
    # results do not depend on the constant-memory chunk size (exact carries)
    t, m, mu, alpha, beta, T = rand_problem(21, 30000, 40, density=0.2, rate=30.0)
    a = run_gpu(H, t, m, mu, alpha, beta, T, 12)
    b = run_gpu(H, t, m, mu, alpha, beta, T, 20)
    assert scalar_rel(a[0], b[0]) < 1e-9
    for x, y in zip(a[1:], b[1:]):
        assert rel_err(x, y) < 1e-7


@pytest.mark.parametrize("M,rows", [(20, 0), (200, 32)])
def test_wide_batches_with_long_gaps(H, M, rows):
    # gaps far longer than 1/beta inside 64-event batches exercise the
    # per-event rescaling path of the dense kernel: the 16-row kernel (M = 20)
    # and the 32-row one (M = 200 with 256-column tiles, set through the
    # launch tuning), whose wide windows add their own events' c_k to u and
    # their pair terms with per-pair decays
    rng = np.random.default_rng(31)
    n = 3000
    gaps = rng.exponential(0.05, size=n)
    gaps[rng.random(n) < 0.05] = 200.0
    t = np.cumsum(gaps)
    m = rng.integers(0, M, size=n).astype(np.int32)
    _, _, mu, alpha, beta, _ = rand_problem(31, 10, M)
    T = float(t[-1] + 0.5)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    try:
        H.set_tuning(dense_cols=256 if rows else 0, dense_rows=rows)
        got = run_gpu(H, t, m, mu, alpha, beta, T)
    finally:
        H.set_tuning()
    check(got, ref, label=f"wide M={M} rows={rows or 'auto'}")


def test_determinism_bitwise(H):
    # every result is bitwise repeatable except the large-M engine's
    # dL/dalpha, whose dense kernel lets two waves add into one LDS tile in
    # an order that varies from run to run (rounding-level differences)
    t, m, mu, alpha, beta, T = rand_problem(41, 20000, 50, density=0.2, rate=30.0)
    a = run_gpu(H, t, m, mu, alpha, beta, T)
    b = run_gpu(H, t, m, mu, alpha, beta, T)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
    assert rel_err(a[2], b[2]) < 1e-13
    t, m, mu, alpha, beta, T = rand_problem(42, 20000, 6, rate=3.0)
    a = run_gpu(H, t, m, mu, alpha, beta, T)
    b = run_gpu(H, t, m, mu, alpha, beta, T)
    assert a[0] == b[0] and all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))


# ------------------------------------------------------------- per-record decays in the forward pass
# A segment of 1024 events whose span times beta exceeds 600 would overflow
# the anchored records (e^{beta u} past float64 range), so its records keep
# their own times and are decayed on use.  Rate 1 with beta >= 1 makes every
# segment such a one; a sequence alternating rate-1 and rate-40 stretches
# mixes both forms across the segments of one chunk.  The gradient, the
# loglik-only and the intensity forms of the forward pass are checked.
@pytest.mark.parametrize("mixed", [False, True])
def test_large_engine_per_record_decays(H, mixed):
    import torch
    n, M = 9000, 40
    t, m, mu, alpha, beta, T = rand_problem(91 + mixed, n, M, density=0.3, rate=1.0)
    beta = np.array([1.25], np.float32)
    if mixed:
        rng = np.random.default_rng(93)
        gaps = np.concatenate([rng.exponential(1.0 if (k // 1024) % 2 == 0 else 1.0 / 40.0, 1024)
                               for k in range(0, n, 1024)])[:n]
        t = np.cumsum(gaps)
        T = float(t[-1] + 0.5)
    spans = [float(beta[0]) * (t[min(k + 1023, n - 1)] - t[max(k - 1, 0)]) for k in range(0, n, 1024)]
    assert max(spans) > 600.0 and (not mixed or min(spans) < 600.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T, 12), ref, label=f"per-record decays mixed={mixed}")
    args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
            dev(beta, torch.float32), T)
    assert scalar_rel(H.loglik(*args, 12).item(), ref[0]) < TOL
    lam = H.intensity(*args, 12).cpu().numpy()
    idx = np.unique(np.linspace(0, n - 1, 80).astype(np.int64))
    lref = oracle.intensity_at(t, m, mu, alpha, beta, idx)
    assert np.max(np.abs(lam[idx] - lref) / lref) < 1e-6


# ------------------------------------------------------------- intensities and loglik-only
@pytest.mark.parametrize("M", [1, 6, 40])
def test_intensity_matches_definition(H, M):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(51 + M, 4000, M, density=0.3 if M > 8 else 1.0, rate=10.0)
    lam = H.intensity(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                      dev(alpha, torch.float32), dev(beta, torch.float32), T).cpu().numpy()
    idx = np.unique(np.concatenate([np.arange(5), np.linspace(0, 3999, 60).astype(np.int64)]))
    ref = oracle.intensity_at(t, m, mu, alpha, beta, idx)
    err = np.max(np.abs(lam[idx] - ref) / ref)
    print(f"intensity M={M} max rel err {err:.2e}", flush=True)
    assert err < 1e-6


@pytest.mark.parametrize("M", [2, 30])
def test_loglik_only_matches(H, M):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(61 + M, 8000, M, density=0.5, rate=10.0)
    L = H.loglik(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                 dev(beta, torch.float32), T).item()
    Lr = oracle.forward(t, m, mu, alpha, beta, T, grad=False)
    assert scalar_rel(L, Lr) < TOL


# ------------------------------------------------------------- shared decay above 64 KiB of LDS
# The shared-decay forward kernel keeps 24 bytes of LDS per node, so from
# M = 2731 on it runs under the device's larger per-workgroup limit (160 KiB
# on MI355X, less the kernel's own 2 KiB of static LDS: M <= 6741); one node
# more is refused on the host, before any launch.
def test_shared_decay_above_64k_lds(H):
    t, m, mu, alpha, beta, T = rand_problem(71, 12000, 2600, density=0.002, rate=20.0)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(run_gpu(H, t, m, mu, alpha, beta, T), ref, label="large n=12000 M=2600")


def test_shared_decay_node_limit(H):
    import torch
    for M, ok in ((6741, True), (6742, False)):
        t, m, mu, alpha, beta, T = rand_problem(72, 3000, M, density=0.001, rate=20.0)
        args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                dev(beta, torch.float32), T)
        if ok:
            L = H.loglik(*args).item()
            assert scalar_rel(L, oracle.forward(t, m, mu, alpha, beta, T, grad=False)) < TOL
        else:
            with pytest.raises(H.HawkesError) as e:
                H.loglik(*args)
            assert e.value.status == 4
    # a refusal leaves no pending runtime error behind: a fresh device
    # allocation and a call at a supported size both still succeed
    torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    t, m, mu, alpha, beta, T = rand_problem(74, 2000, 30, density=0.5, rate=10.0)
    L = H.loglik(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                 dev(beta, torch.float32), T).item()
    assert scalar_rel(L, oracle.forward(t, m, mu, alpha, beta, T, grad=False)) < TOL


# ------------------------------------------------------------- paper workloads, reduced sizes
def test_c1_univariate_vs_bruteforce(H):
    from paper_2604_01342_amd import workloads as W
    w = W.make_config(1)
    Lb = oracle.brute(w.t, w.m, w.mu, w.alpha, w.beta, w.T, grad=False)
    gpu = run_gpu(H, w.t, w.m, w.mu, w.alpha, w.beta, w.T)
    print(f"c1 N={w.n}: L_gpu {gpu[0]:.10f} L_brute {Lb:.10f} rel {scalar_rel(gpu[0], Lb):.2e}", flush=True)
    assert scalar_rel(gpu[0], Lb) < TOL
    check(gpu, oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T), label="c1")


def test_c2_reduced(H):
    from paper_2604_01342_amd import workloads as W
    w = W.make_config(2, n=100_000)
    check(run_gpu(H, w.t, w.m, w.mu, w.alpha, w.beta, w.T), oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T),
          label="c2 n=1e5")


def test_c4_reduced(H):
    from paper_2604_01342_amd import workloads as W
    w = W.make_config(4, n=200_000)
    check(run_gpu(H, w.t, w.m, w.mu, w.alpha, w.beta, w.T), oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T),
          label="c4 n=2e5")


def test_c4_reduced_perturbed_theta(H):
    # gradient gate at theta_pert = (1.25 mu, 0.8 alpha, 1.2 beta)
    from paper_2604_01342_amd import workloads as W
    w = W.make_config(4, n=200_000)
    mu = (1.25 * w.mu).astype(np.float32)
    al = (0.8 * w.alpha).astype(np.float32)
    be = (1.2 * w.beta).astype(np.float32)
    check(run_gpu(H, w.t, w.m, mu, al, be, w.T), oracle.forward(w.t, w.m, mu, al, be, w.T), label="c4 pert")


# ------------------------------------------------------------- batched
def _batch(S, max_len, seed=3002):
    from paper_2604_01342_amd import workloads as W
    return W.make_batched(S=S, lo=100, hi=100_000, seed=seed, max_len=max_len)


def test_batched_matches_oracle_per_sequence(H):
    import torch
    bw = _batch(40, 3000)
    b = H.Batch.from_numpy(bw)
    ll, gmu, ga, gb = H.loglik_grad_batched(b)
    torch.cuda.synchronize()
    ll, gmu, ga, gb = ll.cpu().numpy(), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()
    mo = ao = 0
    worst = 0.0
    for s in range(bw.S):
        w = bw.seq(s)
        M = w.M
        ref = oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T)
        e = check((ll[s], gmu[mo:mo + M], ga[ao:ao + M * M].reshape(M, M), gb[s:s + 1]), ref, label=f"seq {s}")
        worst = max(worst, max(e))
        mo += M
        ao += M * M
    print(f"batched worst {worst:.2e}")


def test_batched_graph_replays_equal_eager_calls(H):
    # the batched call captured in a HIP graph: every replay (with eager
    # calls and synchronizations between them) gives the eager result bit
    # for bit, and values written into the batch in place are picked up
    import torch
    bw = _batch(20, 4000, seed=5)
    b = H.Batch.from_numpy(bw)
    eager = [x.clone() for x in H.loglik_grad_batched(b)]
    g = H.BatchedGraph(b)
    for _ in range(3):
        H.loglik_grad_batched(b)
        torch.cuda.synchronize()
        got = g.replay()
        torch.cuda.synchronize()
        for x, e in zip(got, eager):
            assert torch.equal(x, e)
    b.mu.mul_(1.1)
    eager2 = [x.clone() for x in H.loglik_grad_batched(b)]
    got = g.replay()
    torch.cuda.synchronize()
    for x, e in zip(got, eager2):
        assert torch.equal(x, e)
    assert not torch.equal(eager2[0], eager[0])


def test_batched_equals_single_calls(H):
    import torch
    bw = _batch(12, 5000, seed=77)
    b = H.Batch.from_numpy(bw)
    ll, gmu, ga, gb = [x.cpu().numpy() for x in H.loglik_grad_batched(b)]
    mo = ao = 0
    for s in range(bw.S):
        w = bw.seq(s)
        M = w.M
        single = run_gpu(H, w.t, w.m, w.mu, w.alpha, w.beta, w.T)
        assert scalar_rel(ll[s], single[0]) < 1e-12
        assert rel_err(gmu[mo:mo + M], single[1]) < 1e-12
        assert rel_err(ga[ao:ao + M * M], single[2].ravel()) < 1e-12
        mo += M
        ao += M * M


def test_batched_loglik_only(H):
    bw = _batch(20, 2000, seed=5)
    b = H.Batch.from_numpy(bw)
    ll = H.loglik_batched(b).cpu().numpy()
    for s in range(bw.S):
        w = bw.seq(s)
        assert scalar_rel(ll[s], oracle.forward(w.t, w.m, w.mu, w.alpha, w.beta, w.T, grad=False)) < TOL


# ------------------------------------------------------------- baseline kernel, checks, autograd
@pytest.mark.parametrize("M", [1, 12, 100])
def test_sequential_baseline_matches_oracle(H, M):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(71 + M, 2000, M, density=0.3, rate=5.0)
    g = H.sequential_loglik_grad(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                                 dev(alpha, torch.float32), dev(beta, torch.float32), T)
    torch.cuda.synchronize()
    check((g[0].item(), g[1].cpu().numpy(), g[2].cpu().numpy(), g[3].cpu().numpy()),
          oracle.forward(t, m, mu, alpha, beta, T), label=f"sequential M={M}")


def test_check_inputs_flags(H):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(81, 500, 10)
    args = lambda t_, m_, mu_, a_, b_, T_: H.check_inputs(dev(t_, torch.float64), dev(m_, torch.int32),
                                                         dev(mu_, torch.float32), dev(a_, torch.float32),
                                                         dev(b_, torch.float32), T_)
    assert args(t, m, mu, alpha, beta, T) == 0
    t2 = t.copy(); t2[100], t2[101] = t2[101], t2[100] - 1.0
    assert args(t2, m, mu, alpha, beta, T) & 1
    m2 = m.copy(); m2[7] = 10
    assert args(t, m2, mu, alpha, beta, T) & 2
    assert args(t, m, mu, alpha, beta, float(t[-1] - 1.0)) & 4
    mu2 = mu.copy(); mu2[3] = 0.0
    assert args(t, m, mu2, alpha, beta, T) & 8
    a2 = alpha.copy(); a2[2, 2] = -0.1
    assert args(t, m, mu, a2, beta, T) & 16
    assert args(t, m, mu, alpha, -beta, T) & 32


def test_autograd_function(H):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(91, 3000, 12, density=0.5, rate=10.0)
    mu_t = dev(mu, torch.float32).requires_grad_()
    a_t = dev(alpha, torch.float32).requires_grad_()
    b_t = dev(beta, torch.float32).requires_grad_()
    L = H.hawkes_loglik(dev(t, torch.float64), dev(m, torch.int32), mu_t, a_t, b_t, T)
    (2.0 * L).backward()
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    assert scalar_rel(L.item(), ref[0]) < TOL
    assert rel_err(mu_t.grad.cpu().numpy(), 2 * ref[1]) < 1e-6
    assert rel_err(a_t.grad.cpu().numpy(), 2 * ref[2][0]) < 1e-6
    assert rel_err(b_t.grad.cpu().numpy(), 2 * ref[3]) < 1e-6
