"""GPU parity at launch configurations that only large inputs or uneven
batches reach.

* Chunks longer than 2^20 events (chunk_log2 = 24, 25, 26): the dense
  dL/dalpha kernel then takes 256-, 128- and 64-column tiles whose record
  keys (index in chunk << bits of the local mark) reach bit 31 of their
  32-bit word, and its checkpoint slots hold up to 1.7 GB addressed with
  32-bit offsets.  Each case has a full chunk and a ragged second one.
* Batches whose sequences differ in node count (1..8) and length (0..1e4):
  the device-side packing of each sequence's parameters and outputs; and
  batches with larger sequences (up to 100 nodes), which the library splits
  between its small-M and large-M engines.

Every result is compared with the FP64 oracle (oracle.forward) at 1e-6
relative, per sequence for batches.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import rand_batch, rand_problem, rel_err, scalar_rel

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01342_amd as H
    H.lib()
    H.set_tuning()
    return H


def dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def check(gpu, ref, label):
    L, gmu, ga, gb = gpu
    Lr, gmur, gar, gbr = ref
    errs = (scalar_rel(L, Lr), rel_err(gmu, gmur), rel_err(ga, np.reshape(gar, np.shape(ga))),
            rel_err(gb, np.ravel(gbr)))
    print(f"{label}: L {errs[0]:.2e} mu {errs[1]:.2e} alpha {errs[2]:.2e} beta {errs[3]:.2e}", flush=True)
    for name, e in zip(("loglik", "g_mu", "g_alpha", "g_beta"), errs):
        assert e <= TOL, f"{label}: {name} rel err {e}"
    return errs


# (chunk_log2, M): 256-column tiles need chunk_log2 <= 24, 128 <= 25, 64 <= 26;
# M is chosen so that the rule keeps the widest tile the chunk allows
@pytest.mark.timeout(400)
@pytest.mark.parametrize("lg,M", [(24, 256), (25, 100), (26, 70)])
def test_long_chunks_match_oracle(H, lg, M):
    import torch
    n = (1 << lg) + (1 << (lg - 2)) + 12345   # one full chunk, one ragged
    print(f"long chunk case: chunk_log2={lg} M={M} n={n}", flush=True)
    t, m, mu, alpha, beta, T = rand_problem(900 + lg, n, M, density=0.2, rate=40.0)
    args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
            dev(beta, torch.float32))
    L, gmu, ga, gb = H.loglik_grad(*args, T, lg)
    torch.cuda.synchronize()
    gpu = (float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy())
    del args, L, gmu, ga, gb
    torch.cuda.empty_cache()
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(gpu, ref, f"chunk_log2={lg} M={M} n={n}")


# The 32-row dense kernel adds its float32 rank-1 accumulators to the float64
# tile every 256 windows that had own events.  At c4's shape a wave visits
# about 150 windows per launch, so there only the final flush runs; here one
# event range per chunk (the launch tuning) gives each of a tile's four waves
# a quarter of a 2^20-event chunk, about 1300 windows with own events at
# M = 400, so the periodic flush runs several times per wave.
@pytest.mark.timeout(300)
def test_dense_float32_accumulators_flush_periodically(H):
    import torch
    M, n = 400, (1 << 20) + 54321
    print(f"periodic flush case: M={M} n={n} one event range", flush=True)
    t, m, mu, alpha, beta, T = rand_problem(951, n, M, density=0.05, rate=60.0)
    args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
            dev(beta, torch.float32))
    try:
        H.set_tuning(dense_ranges=1, dense_rows=32)
        L, gmu, ga, gb = H.loglik_grad(*args, T, 20)
        torch.cuda.synchronize()
    finally:
        H.set_tuning()
    gpu = (float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy())
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(gpu, ref, f"periodic flush M={M} n={n}")


def _batch_to_dev(H, pb):
    import torch
    return H.Batch(dev(pb.ev_off, torch.int64), dev(pb.m_s, torch.int32), dev(pb.T_s, torch.float64),
                   dev(pb.t, torch.float64), dev(pb.m, torch.int32), dev(pb.mu, torch.float32),
                   dev(pb.alpha, torch.float32), dev(pb.beta, torch.float32), int(pb.m_s.max()))


def _check_batch(pb, out, label):
    ll, gmu, ga, gb = [x.cpu().numpy() for x in out]
    worst = 0.0
    for s in range(pb.S):
        t, m, mu, alpha, beta, T = pb.seq(s)
        M = int(pb.m_s[s])
        ref = oracle.forward(t, m, mu, alpha, beta, T)
        got = (ll[s], gmu[pb.mu_off[s]:pb.mu_off[s + 1]],
               ga[pb.a_off[s]:pb.a_off[s + 1]].reshape(M, M), gb[s:s + 1])
        errs = (scalar_rel(got[0], ref[0]), rel_err(got[1], ref[1]), rel_err(got[2], ref[2]),
                rel_err(got[3], np.ravel(ref[3])) if len(t) else abs(float(got[3][0])))
        for name, e in zip(("loglik", "g_mu", "g_alpha", "g_beta"), errs):
            assert e <= TOL, f"{label} sequence {s} (M={M}, n={len(t)}): {name} rel err {e}"
        worst = max(worst, max(errs))
    print(f"{label}: {pb.S} sequences, worst {worst:.2e}", flush=True)


def test_batch_with_mixed_node_counts(H):
    # node counts 1..8 and lengths 0..1e4 in one batch, every sequence
    # checked; then the same batch from a HIP graph, replayed between eager
    # calls, bit for bit
    import torch
    pb = rand_batch(4242, 160, list(range(1, 9)), lo=1, hi=10_000, n_empty=3)
    b = _batch_to_dev(H, pb)
    eager = [x.clone() for x in H.loglik_grad_batched(b)]
    torch.cuda.synchronize()
    _check_batch(pb, eager, "mixed M batch")
    g = H.BatchedGraph(b)
    for _ in range(3):
        H.loglik_grad_batched(b)
        torch.cuda.synchronize()
        got = g.replay()
        torch.cuda.synchronize()
        for x, e in zip(got, eager):
            assert torch.equal(x, e)
    ll = H.loglik_batched(b).cpu().numpy()
    for s in range(pb.S):
        assert scalar_rel(ll[s], float(eager[0][s])) <= 1e-12


def test_batched_graph_keeps_its_workspace(H):
    # a larger call after capture grows the module's shared workspace; the
    # graph's kernels point into the graph's own workspace, so replays still
    # equal an eager call
    import torch
    pb = rand_batch(99, 40, [2, 5, 8], lo=10, hi=3000)
    b = _batch_to_dev(H, pb)
    g = H.BatchedGraph(b)
    eager = [x.clone() for x in H.loglik_grad_batched(b)]
    t, m, mu, alpha, beta, T = rand_problem(5, 300_000, 300, density=0.1, rate=20.0)
    H.loglik_grad(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
                  dev(beta, torch.float32), T)
    filler = [torch.full((1 << 20,), 7.0, dtype=torch.float64, device="cuda") for _ in range(8)]
    torch.cuda.synchronize()
    got = g.replay()
    torch.cuda.synchronize()
    for x, e in zip(got, eager):
        assert torch.equal(x, e)
    assert all(bool((f == 7.0).all()) for f in filler)


def test_batch_with_large_node_counts(H):
    # node counts 1..100 in one batch (sequences above 8 nodes go through the
    # large-M engine one by one), every sequence checked against the oracle;
    # the log-likelihood-only call agrees; such a batch cannot be captured
    import torch
    pb = rand_batch(777, 48, [1, 3, 8, 9, 16, 33, 64, 100], lo=1, hi=8000, n_empty=2, rate=10.0)
    b = _batch_to_dev(H, pb)
    assert b.max_m == 100
    out = H.loglik_grad_batched(b)
    torch.cuda.synchronize()
    _check_batch(pb, out, "batch with M up to 100")
    ll = H.loglik_batched(b).cpu().numpy()
    for s in range(pb.S):
        assert scalar_rel(ll[s], float(out[0][s])) <= 1e-12
    with pytest.raises(ValueError):
        H.BatchedGraph(b)
