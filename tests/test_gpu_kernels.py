"""GPU parity with several decay kernels (Background, eq. 1 with K > 1;
gradients per kernel, eqs. 8-10; the paper's studies use K = 3).

alpha is K x M x M and beta holds one decay per kernel, shared by every
node.  The library runs its large-M engine once per kernel for the states
and the dense dL/dalpha, with the intensities, 1/lambda and the
log-likelihood formed from all kernels together.  Every result is compared
with the FP64 oracle (oracle.forward, K kernels) at 1e-6 relative, per
gradient block (normwise over all kernels, and per kernel).
"""
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
    H.set_tuning()
    return H


def dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def multi_problem(seed, n, M, K, density=1.0, rate=20.0, rho=0.6):
    """Random sorted events; K interaction matrices whose summed column sums
    stay below rho; decays spread over a decade (fast, medium, slow)."""
    t, m, mu, _, _, T = rand_problem(seed, n, M, rate=rate)
    rng = np.random.default_rng(seed + 7)
    a = rng.uniform(0.0, 1.0, size=(K, M, M))
    if density < 1.0:
        a *= rng.random((K, M, M)) < density
    s = a.sum(axis=(0, 1)).max()
    alpha = (a * (rho / s if s > 0 else 1.0)).astype(np.float32)
    beta = (np.array([3.0, 1.0, 0.3, 2.0, 0.6, 5.0, 0.15, 1.5])[:K] * rng.uniform(0.8, 1.25, size=K)).astype(
        np.float32)
    return t, m, mu, alpha, beta, T


def run(H, t, m, mu, alpha, beta, T, chunk=0, support=False):
    import torch
    L, gmu, ga, gb = H.loglik_grad(dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32),
                                   dev(alpha, torch.float32), dev(beta, torch.float32), T, chunk, support=support)
    torch.cuda.synchronize()
    return float(L.item()), gmu.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()


def check(got, ref, K, label):
    L, gmu, ga, gb = got
    Lr, gmur, gar, gbr = ref
    ga = np.reshape(ga, (K, -1))
    gar = np.reshape(gar, (K, -1))
    errs = {"loglik": scalar_rel(L, Lr), "g_mu": rel_err(gmu, gmur), "g_alpha": rel_err(ga, gar),
            "g_beta": rel_err(gb, np.ravel(gbr))}
    for k in range(K):
        errs[f"g_alpha[{k}]"] = rel_err(ga[k], gar[k])
        errs[f"g_beta[{k}]"] = scalar_rel(gb[k], np.ravel(gbr)[k])
    print(f"{label}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for name, e in errs.items():
        assert e <= TOL, f"{label}: {name} rel err {e}"


# M = 1 and 8 take the large-M engine too when K > 1; chunk 12 puts several
# chunk boundaries inside the sequence
@pytest.mark.parametrize("K,M,n,density,chunk", [(2, 1, 9000, 1.0, 12), (3, 1, 3000, 1.0, 0),
                                                 (2, 8, 12000, 1.0, 12), (3, 8, 5000, 1.0, 0),
                                                 (2, 40, 20000, 0.3, 12), (3, 40, 9000, 0.3, 0),
                                                 (2, 1000, 30000, 0.01, 12), (3, 1000, 40000, 0.01, 0),
                                                 (3, 300, 25000, 0.05, 13), (8, 20, 6000, 0.5, 12)])
def test_kernels_match_oracle(H, K, M, n, density, chunk):
    print(f"K={K} M={M} n={n} chunk={chunk}", flush=True)
    t, m, mu, alpha, beta, T = multi_problem(100 * K + M, n, M, K, density=density)
    ref = oracle.forward(t, m, mu, alpha, beta, T)
    check(run(H, t, m, mu, alpha, beta, T, chunk), ref, K, f"K={K} M={M} n={n} chunk={chunk}")


def test_one_kernel_split_in_two_equals_one(H):
    # alpha split into two kernels with the same decay: the same model, so the
    # log-likelihood and dL/dmu equal the one-kernel call's, and each kernel's
    # dL/dalpha equals the one-kernel dL/dalpha
    t, m, mu, alpha, beta, T = rand_problem(55, 15000, 60, density=0.2, rate=25.0)
    a2 = np.stack([alpha * np.float32(0.25), alpha * np.float32(0.75)])
    b2 = np.repeat(beta, 2)
    one = run(H, t, m, mu, alpha, beta, T)
    two = run(H, t, m, mu, a2, b2, T)
    assert scalar_rel(two[0], one[0]) < 1e-7
    assert rel_err(two[1], one[1]) < 1e-7
    for k in range(2):
        assert rel_err(two[2][k], one[2]) < 1e-6


def test_kernels_loglik_intensity_support(H):
    import torch
    K, M = 3, 50
    t, m, mu, alpha, beta, T = multi_problem(77, 12000, M, K, density=0.2)
    args = (dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
            dev(beta, torch.float32))
    Lr, gmur, gar, gbr = oracle.forward(t, m, mu, alpha, beta, T)
    L = float(H.loglik(*args, T, 12).item())
    assert scalar_rel(L, Lr) <= TOL
    lam = H.intensity(*args, T, 12).cpu().numpy()
    idx = np.array([0, 1, 57, 4095, 4096, 8191, 11999], dtype=np.int64)
    lam_ref = oracle.intensity_at(t, m, mu, alpha, beta, idx)
    assert rel_err(lam[idx], lam_ref) <= TOL
    # support-restricted gradient: the dense one, zero off alpha's support
    got = run(H, t, m, mu, alpha, beta, T, 12, support=True)
    gmask = np.where(alpha != 0.0, np.reshape(gar, alpha.shape), 0.0)
    check(got, (Lr, gmur, gmask, gbr), K, "K=3 support")
    assert np.all(np.reshape(got[2], alpha.shape)[alpha == 0.0] == 0.0)


def test_kernels_check_inputs(H):
    import torch
    K, M = 2, 12
    t, m, mu, alpha, beta, T = multi_problem(3, 100, M, K)
    args = [dev(t, torch.float64), dev(m, torch.int32), dev(mu, torch.float32), dev(alpha, torch.float32),
            dev(beta, torch.float32)]
    assert H.check_inputs(*args, T) == 0
    bad = beta.copy()
    bad[1] = -1.0
    args[4] = dev(bad, torch.float32)
    assert H.check_inputs(*args, T) == 32
    bada = alpha.copy()
    bada[1, 3, 4] = -0.5
    args[4] = dev(beta, torch.float32)
    args[3] = dev(bada, torch.float32)
    assert H.check_inputs(*args, T) == 16


def test_kernels_empty_sequence(H):
    import torch
    K, M = 3, 10
    mu = np.full(M, 0.3, np.float32)
    alpha = np.full((K, M, M), 0.01, np.float32)
    beta = np.array([0.5, 1.0, 2.0], np.float32)
    L, gmu, ga, gb = run(H, np.zeros(0), np.zeros(0, np.int32), mu, alpha, beta, 2.0)
    assert L == pytest.approx(-2.0 * float(mu.astype(np.float64).sum()), rel=1e-12)
    np.testing.assert_allclose(gmu, -2.0)
    np.testing.assert_allclose(ga, 0.0)
    np.testing.assert_allclose(gb, 0.0)
