"""hawkes_loglik_grad_noalloc (the entry point for callers that cannot
allocate): its output equals hawkes_loglik_grad's on the same inputs, on
consecutive calls that share the library's fixed scratch (a larger problem,
then smaller ones, so that stale scratch contents would show), and problems
whose workspace exceeds the scratch are refused before any launch."""
import numpy as np
import pytest

import oracle
from tests.helpers import rand_problem, rel_err, scalar_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01342_amd as H
    H.lib()
    H.set_tuning()
    return H


def _dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _inputs(seed, n, M, per_target=False, density=1.0, rate=20.0, chunk=0):
    import torch
    t, m, mu, alpha, beta, T = rand_problem(seed, n, M, per_target=per_target, density=density, rate=rate)
    d = (_dev(t, torch.float64), _dev(m, torch.int32), _dev(mu, torch.float32), _dev(alpha, torch.float32),
         _dev(beta, torch.float32))
    return (t, m, mu, alpha, beta, T), d, T, chunk


def _host(x):
    L, gmu, ga, gb = x
    return float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()


# a larger problem first, then smaller ones on the same scratch: large-M
# shared decay, small-M, per-target decays, a second large-M call
CASES = [(1, 200_000, 150, False, 0.05, 30.0, 0), (2, 7_000, 40, False, 0.3, 20.0, 12),
         (3, 20_000, 6, False, 1.0, 3.0, 0), (4, 9_000, 30, True, 0.3, 5.0, 0),
         (5, 3_000, 12, False, 1.0, 10.0, 0)]


def test_noalloc_equals_loglik_grad_on_consecutive_calls(H):
    import torch
    for seed, n, M, pt, dens, rate, chunk in CASES:
        print(f"noalloc case seed={seed} n={n} M={M} per_target={pt} chunk={chunk}", flush=True)
        host, d, T, chunk = _inputs(seed, n, M, pt, dens, rate, chunk)
        assert H.workspace_bytes(n, M, per_target=pt, grad=True, chunk_log2=chunk) <= H.NOALLOC_SCRATCH_BYTES
        got = _host(H.loglik_grad_noalloc(*d, T, chunk))
        ref = _host(H.loglik_grad(*d, T, chunk))
        torch.cuda.synchronize()
        # the same kernels on the same inputs: equal up to the last-bit
        # variation of the large-M dL/dalpha sums (LDS atomics of several waves)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1])
        assert rel_err(got[2], ref[2]) <= 1e-12
        assert np.array_equal(got[3], ref[3])
        orc = (oracle.adjoint if pt else oracle.forward)(*host)
        errs = (scalar_rel(got[0], orc[0]), rel_err(got[1], orc[1]), rel_err(got[2], np.reshape(orc[2], (M, M))),
                rel_err(got[3], np.ravel(orc[3])))
        print(f"  vs oracle: {errs}", flush=True)
        assert max(errs) <= 1e-6


def test_noalloc_refuses_problems_beyond_the_scratch(H):
    # a valid problem (inputs of the stated size) whose workspace exceeds the
    # scratch: refused before any launch, outputs untouched
    import torch
    n, M = 3_000_000, 1000
    host, d, T, _ = _inputs(9, n, M, density=0.01)
    assert H.workspace_bytes(n, M, grad=True) > H.NOALLOC_SCRATCH_BYTES
    out = (torch.full((1,), -5.0, dtype=torch.float64, device="cuda"),
           torch.full((M,), -5.0, dtype=torch.float64, device="cuda"),
           torch.full((M, M), -5.0, dtype=torch.float64, device="cuda"),
           torch.full((1,), -5.0, dtype=torch.float64, device="cuda"))
    with pytest.raises(H.HawkesError) as e:
        H.loglik_grad_noalloc(*d, T, 0, out=out)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert all(bool((x == -5.0).all()) for x in out)
