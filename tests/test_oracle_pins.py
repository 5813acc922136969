"""Pins of the FP64 oracle to things other than itself.

Every expected value here comes from the paper's definitions (eq. 1 intensity,
eq. 2 log-likelihood, eqs. 8-10 gradients) written out in closed form for tiny
inputs, from textbook special cases, from brute force on tiny inputs, from
finite differences, or from exact invariants of the model.  A dropped term, a
wrong sign or index, or a transposed alpha makes at least one of them fail.
"""
import math

import numpy as np
import pytest

import oracle


def rand_problem(rng, n, M, K=1, per_target=False, ties=False, scale=1.0):
    gaps = rng.exponential(scale, size=n)
    if ties and n > 3:
        gaps[rng.random(n) < 0.2] = 0.0
    t = np.cumsum(gaps)
    m = rng.integers(0, M, size=n).astype(np.int32)
    mu = rng.uniform(0.2, 1.0, size=M)
    alpha = rng.uniform(0.0, 0.6, size=(K, M, M)) / M
    if per_target:
        beta = rng.uniform(0.5, 2.0, size=M)
    else:
        beta = rng.uniform(0.5, 2.0, size=K)
    T = (t[-1] if n else 0.0) + rng.uniform(0.0, 2.0)
    return t, m, mu, alpha, beta, T


# ---------------------------------------------------------------- closed forms
def hand_two_events(mu, a, b, T):
    """M=1, events at t=1 and t=2 (eq. 1 and eq. 2 written out)."""
    l1 = mu
    l2 = mu + a * b * math.exp(-b)
    L = math.log(l1) + math.log(l2) - mu * T - a * ((1 - math.exp(-b * (T - 1))) + (1 - math.exp(-b * (T - 2))))
    gmu = 1 / l1 + 1 / l2 - T
    ga = b * math.exp(-b) / l2 - (1 - math.exp(-b * (T - 1))) - (1 - math.exp(-b * (T - 2)))
    gb = a * (1 - b) * math.exp(-b) / l2 - a * ((T - 1) * math.exp(-b * (T - 1)) + (T - 2) * math.exp(-b * (T - 2)))
    return L, gmu, ga, gb


@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_hand_example(fn):
    t = np.array([1.0, 2.0]); m = np.array([0, 0])
    L, gmu, ga, gb = getattr(oracle, fn)(t, m, [0.5], [[0.5]], [1.0], 3.0)
    eL, emu, ea, eb = hand_two_events(0.5, 0.5, 1.0, 3.0)
    assert L == pytest.approx(eL, rel=1e-14, abs=1e-14)
    assert gmu[0] == pytest.approx(emu, rel=1e-13)
    assert np.ravel(ga)[0] == pytest.approx(ea, rel=1e-13)
    assert np.ravel(gb)[0] == pytest.approx(eb, rel=1e-13)
    # printed values of the same closed form, for the record
    assert eL == pytest.approx(-3.32142531139764, abs=1e-13)
    assert eb == pytest.approx(-0.31927500382233, abs=1e-13)


@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_hand_other_parameters(fn):
    L, gmu, ga, gb = getattr(oracle, fn)(np.array([1.0, 2.0]), np.array([0, 0]), [0.3], [[0.7]], [2.5], 4.0)
    eL, emu, ea, eb = hand_two_events(0.3, 0.7, 2.5, 4.0)
    assert L == pytest.approx(eL, rel=1e-13)
    assert (gmu[0], np.ravel(ga)[0], np.ravel(gb)[0]) == pytest.approx((emu, ea, eb), rel=1e-12)


@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_single_event(fn):
    L = getattr(oracle, fn)(np.array([1.0]), np.array([0]), [0.5], [[0.5]], [1.0], 3.0, grad=False)
    assert L == pytest.approx(math.log(0.5) - 1.5 - 0.5 * (1 - math.exp(-2.0)), rel=1e-14)
    assert L == pytest.approx(-2.62547953894164, abs=1e-13)


@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_tied_times_follow_index_order(fn):
    # two events at the same instant: the second is excited by the first
    mu, a, b, T = 0.4, 0.3, 1.7, 2.0
    L = getattr(oracle, fn)(np.array([1.0, 1.0]), np.array([0, 0]), [mu], [[a]], [b], T, grad=False)
    e = math.log(mu) + math.log(mu + a * b) - mu * T - 2 * a * (1 - math.exp(-b * (T - 1)))
    assert L == pytest.approx(e, rel=1e-14)


def test_alpha_orientation_target_source():
    # eq. 1: lambda_p uses alpha[p, m_j]; node 0 excites node 1 only.
    mu = np.array([0.2, 0.3]); alpha = np.zeros((2, 2)); alpha[1, 0] = 0.8
    beta = np.array([1.5])
    t = np.array([0.5, 0.9, 1.4]); m = np.array([0, 1, 0])
    lam = oracle.intensity_at(t, m, mu, alpha, beta, [0, 1, 2])
    assert lam[0] == pytest.approx(0.2)
    assert lam[1] == pytest.approx(0.3 + 0.8 * 1.5 * math.exp(-1.5 * 0.4), rel=1e-14)
    assert lam[2] == pytest.approx(0.2, rel=1e-14)   # node 1 does not excite node 0
    for fn in ("brute", "forward"):
        L = getattr(oracle, fn)(t, m, mu, alpha, beta, 2.0, grad=False)
        comp = 0.5 * 2.0 + 0.8 * ((1 - math.exp(-1.5 * 1.5)) + (1 - math.exp(-1.5 * 0.6)))
        assert L == pytest.approx(np.log(lam).sum() - comp, rel=1e-14)
    La = oracle.adjoint(t, m, mu, alpha, np.array([1.5, 1.5]), 2.0, grad=False)
    assert La == pytest.approx(L, rel=1e-14)


# ------------------------------------------------------------- special cases
@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_poisson_closed_form(fn):
    rng = np.random.default_rng(4)
    t, m, mu, alpha, beta, T = rand_problem(rng, 200, 4)
    alpha[:] = 0.0
    if fn == "adjoint":
        beta = rng.uniform(0.5, 2, size=4)
    L, gmu, ga, gb = getattr(oracle, fn)(t, m, mu, alpha, beta, T)
    Np = np.bincount(m, minlength=4)
    assert L == pytest.approx(float(np.sum(Np * np.log(mu)) - T * mu.sum()), rel=1e-13)
    np.testing.assert_allclose(gmu, Np / mu - T, rtol=1e-13)
    np.testing.assert_allclose(np.ravel(gb), 0.0, atol=1e-12)


def ozaki_univariate(t, mu, a, b, T):
    """Textbook recursion for the univariate exponential Hawkes process
    (Ozaki 1979): A_i = e^{-b (t_i - t_{i-1})} (1 + A_{i-1}), A_1 = 0."""
    A = 0.0
    L = 0.0
    for i in range(len(t)):
        if i > 0:
            A = math.exp(-b * (t[i] - t[i - 1])) * (1.0 + A)
        L += math.log(mu + a * b * A)
    L -= mu * T
    for ti in t:
        L -= a * (1.0 - math.exp(-b * (T - ti)))
    return L


@pytest.mark.parametrize("fn", ["brute", "forward", "adjoint"])
def test_univariate_textbook_recursion(fn):
    rng = np.random.default_rng(11)
    t, m, mu, alpha, beta, T = rand_problem(rng, 300, 1)
    L = getattr(oracle, fn)(t, m, mu, alpha[0], beta, T, grad=False)
    assert L == pytest.approx(ozaki_univariate(t, mu[0], alpha[0, 0, 0], beta[0], T), rel=1e-13)


def test_empty_sequence():
    mu = np.array([0.2, 0.7]); alpha = np.full((2, 2), 0.1)
    for fn, beta in (("brute", [1.0]), ("forward", [1.0]), ("adjoint", [1.0, 2.0])):
        L, gmu, ga, gb = getattr(oracle, fn)(np.zeros(0), np.zeros(0, np.int32), mu, alpha, beta, 3.0)
        assert L == pytest.approx(-3.0 * 0.9)
        np.testing.assert_allclose(gmu, -3.0)
        np.testing.assert_allclose(np.ravel(ga), 0.0)
        np.testing.assert_allclose(np.ravel(gb), 0.0)


# ---------------------------------------------------- recurrences vs definition
@pytest.mark.parametrize("seed,n,M,K,ties", [(1, 1, 1, 1, False), (2, 2, 3, 1, False), (3, 60, 3, 1, True),
                                             (4, 250, 5, 1, False), (5, 120, 4, 2, True), (6, 400, 2, 3, False)])
def test_forward_equals_brute(seed, n, M, K, ties):
    rng = np.random.default_rng(seed)
    t, m, mu, alpha, beta, T = rand_problem(rng, n, M, K, ties=ties)
    Lb, gmub, gab, gbb = oracle.brute(t, m, mu, alpha, beta, T)
    Lf, gmuf, gaf, gbf = oracle.forward(t, m, mu, alpha, beta, T)
    assert Lf == pytest.approx(Lb, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(gmuf, gmub, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gaf, gab, rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(gbf, gbb.sum(axis=1), rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("seed,n,M,ties", [(21, 1, 1, False), (22, 80, 3, True), (23, 300, 5, False), (24, 200, 6, True)])
def test_adjoint_equals_brute_per_target(seed, n, M, ties):
    rng = np.random.default_rng(seed)
    t, m, mu, alpha, beta, T = rand_problem(rng, n, M, 1, per_target=True, ties=ties)
    Lb, gmub, gab, gbb = oracle.brute(t, m, mu, alpha[0], beta, T)
    La, gmua, gaa, gba = oracle.adjoint(t, m, mu, alpha[0], beta, T)
    assert La == pytest.approx(Lb, rel=1e-12)
    np.testing.assert_allclose(gmua, gmub, rtol=1e-11)
    np.testing.assert_allclose(gaa, gab[0], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(gba, gbb[0], rtol=1e-10, atol=1e-11)


def test_forward_equals_adjoint_shared_beta():
    rng = np.random.default_rng(31)
    t, m, mu, alpha, beta, T = rand_problem(rng, 3000, 7, 1)
    Lf, gmuf, gaf, gbf = oracle.forward(t, m, mu, alpha, beta, T)
    La, gmua, gaa, gba = oracle.adjoint(t, m, mu, alpha[0], np.full(7, beta[0]), T)
    assert La == pytest.approx(Lf, rel=1e-13)
    np.testing.assert_allclose(gmua, gmuf, rtol=1e-12)
    np.testing.assert_allclose(gaa, gaf[0], rtol=1e-10, atol=1e-10)
    assert gba.sum() == pytest.approx(gbf[0], rel=1e-10)


# -------------------------------------------------------- finite differences
def _fd(f, x, i, h):
    xp = x.copy(); xm = x.copy()
    xp.flat[i] += h; xm.flat[i] -= h
    return (f(xp) - f(xm)) / (2 * h)


@pytest.mark.parametrize("per_target", [False, True])
def test_gradients_match_central_differences_of_definition(per_target):
    rng = np.random.default_rng(41 + per_target)
    M = 3
    t, m, mu, alpha, beta, T = rand_problem(rng, 150, M, 1, per_target=per_target)
    a2 = alpha[0]
    fn = oracle.adjoint if per_target else oracle.forward
    L, gmu, ga, gb = fn(t, m, mu, a2, beta, T)
    ga = np.reshape(ga, (M, M)); gb = np.ravel(gb)
    h = 1e-6
    Lb = lambda mu_, a_, b_: oracle.brute(t, m, mu_, a_, b_, T, grad=False)
    for i in range(M):
        assert _fd(lambda x: Lb(x, a2, beta), mu, i, h * mu[i]) == pytest.approx(gmu[i], rel=2e-7, abs=2e-7)
    for i in range(M * M):
        assert _fd(lambda x: Lb(mu, x, beta), a2, i, h) == pytest.approx(ga.flat[i], rel=2e-7, abs=2e-7)
    for i in range(beta.shape[0]):
        assert _fd(lambda x: Lb(mu, a2, x), beta, i, h * beta[i]) == pytest.approx(gb[i], rel=2e-7, abs=2e-7)


def test_two_kernel_gradients_match_central_differences():
    rng = np.random.default_rng(45)
    t, m, mu, alpha, beta, T = rand_problem(rng, 120, 2, K=2)
    L, gmu, ga, gb = oracle.forward(t, m, mu, alpha, beta, T)
    f = lambda a_, b_: oracle.brute(t, m, mu, a_, b_, T, grad=False)
    for i in range(alpha.size):
        assert _fd(lambda x: f(x, beta), alpha, i, 1e-6) == pytest.approx(ga.flat[i], rel=2e-7, abs=2e-7)
    for i in range(2):
        assert _fd(lambda x: f(alpha, x), beta, i, 1e-6 * beta[i]) == pytest.approx(gb[i], rel=2e-7, abs=2e-7)


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("fn", ["forward", "adjoint"])
def test_homogeneity_identity(fn):
    # (mu, alpha) -> c (mu, alpha) scales every intensity by c, so
    # L(c) = L + N log c - (c - 1) Comp, hence sum mu dmu + sum alpha dalpha = N - Comp.
    rng = np.random.default_rng(51)
    M = 4
    t, m, mu, alpha, beta, T = rand_problem(rng, 500, M, 1, per_target=(fn == "adjoint"))
    f = getattr(oracle, fn)
    L, gmu, ga, gb = f(t, m, mu, alpha[0], beta, T)
    L2 = f(t, m, 2 * mu, 2 * alpha[0], beta, T, grad=False)
    comp = t.shape[0] * math.log(2.0) - (L2 - L)
    lhs = float(mu @ gmu + np.sum(alpha[0] * np.reshape(ga, (M, M))))
    assert lhs == pytest.approx(t.shape[0] - comp, rel=1e-11)


@pytest.mark.parametrize("k", [-3, 1, 4])
def test_time_scaling(k):
    c = 2.0 ** k
    rng = np.random.default_rng(61)
    t, m, mu, alpha, beta, T = rand_problem(rng, 400, 3, 2)
    L = oracle.forward(t, m, mu, alpha, beta, T, grad=False)
    Lc = oracle.forward(c * t, m, mu / c, alpha, beta / c, c * T, grad=False)
    assert Lc == pytest.approx(L - t.shape[0] * math.log(c), rel=1e-12)


def test_node_relabelling():
    rng = np.random.default_rng(71)
    M = 5
    t, m, mu, alpha, beta, T = rand_problem(rng, 400, M)
    perm = rng.permutation(M)          # new label of old node q is perm[q]
    inv = np.argsort(perm)
    m2 = perm[m].astype(np.int32)
    mu2 = mu[inv]
    a2 = alpha[0][np.ix_(inv, inv)]
    L, gmu, ga, gb = oracle.forward(t, m, mu, alpha, beta, T)
    L2, gmu2, ga2, gb2 = oracle.forward(t, m2, mu2, a2, beta, T)
    assert L2 == pytest.approx(L, rel=1e-13)
    np.testing.assert_allclose(gmu2, gmu[inv], rtol=1e-12)
    np.testing.assert_allclose(ga2[0], ga[0][np.ix_(inv, inv)], rtol=1e-11, atol=1e-13)
    assert gb2[0] == pytest.approx(gb[0], rel=1e-11)


def test_block_diagonal_independence():
    rng = np.random.default_rng(81)
    t1, m1, mu1, a1, b, _ = rand_problem(rng, 200, 2)
    t2, m2, mu2, a2, _, _ = rand_problem(rng, 300, 3)
    T = max(t1[-1], t2[-1]) + 0.5
    t = np.concatenate([t1, t2]); m = np.concatenate([m1, m2 + 2]).astype(np.int32)
    order = np.argsort(t, kind="stable")
    A = np.zeros((5, 5)); A[:2, :2] = a1[0]; A[2:, 2:] = a2[0]
    L = oracle.forward(t[order], m[order], np.concatenate([mu1, mu2]), A, b, T, grad=False)
    L1 = oracle.forward(t1, m1, mu1, a1, b, T, grad=False)
    L2 = oracle.forward(t2, m2, mu2, a2, b, T, grad=False)
    assert L == pytest.approx(L1 + L2, rel=1e-13)


def test_intensity_at_matches_forward_logsum():
    rng = np.random.default_rng(91)
    t, m, mu, alpha, beta, T = rand_problem(rng, 300, 3, 2)
    lam = oracle.intensity_at(t, m, mu, alpha, beta, np.arange(300))
    L = oracle.forward(t, m, mu, alpha, beta, T, grad=False)
    L0 = oracle.forward(t, m, mu, alpha, beta, t[-1] * 0 + T, grad=False)
    # the log-sum part equals L + Comp; compare through the alpha=0 / mu scaling trick:
    Lb = oracle.brute(t, m, mu, alpha, beta, T, grad=False)
    assert L == pytest.approx(Lb, rel=1e-12)
    comp = float(np.log(lam).sum()) - Lb
    # the compensator of eq. 2 written out
    ec = T * mu.sum() + sum(alpha[k][:, m[j]].sum() * (1 - math.exp(-beta[k] * (T - t[j])))
                            for k in range(2) for j in range(300))
    assert comp == pytest.approx(ec, rel=1e-12)
    assert L0 == L


def test_addend_scales_match_direct_double_sums():
    """The addend split used for errors at the generating point: positive
    parts written out as O(N^2) double sums (eqs. 8-10) on a tiny case."""
    from tests.helpers import rand_problem
    t, m, mu, al, be, T = rand_problem(11, 60, 3)
    L, g_mu, g_a, g_b = oracle.forward(t, m, mu, al, be, T)
    lam = oracle.intensity_at(t, m, mu, al, be, np.arange(len(t)))
    w = 1.0 / lam
    b = float(be[0])
    M = len(mu)
    S = np.array([w[m == p].sum() for p in range(M)])
    G = np.zeros((M, M))
    Gb = 0.0
    a = np.asarray(al, dtype=np.float64).reshape(M, M)
    for i in range(len(t)):
        for j in range(i):
            e = np.exp(-b * (t[i] - t[j]))
            G[m[i], m[j]] += b * w[i] * e
            Gb += w[i] * a[m[i], m[j]] * e * (1.0 - b * (t[i] - t[j]))
    C = np.array([np.sum(-np.expm1(-b * (T - t[m == q]))) for q in range(M)])
    E = float(np.sum(a.sum(axis=0)[m] * (T - t) * np.exp(-b * (T - t))))
    s_mu, s_a, s_b = oracle.addend_scales(t, m, mu, al, be, T, (g_mu, g_a, g_b))
    assert abs(s_mu - np.linalg.norm(S + T)) <= 1e-12 * s_mu
    assert abs(s_a - np.linalg.norm(G + C[None, :])) <= 1e-12 * s_a
    assert abs(s_b - (abs(Gb) + E)) <= 1e-12 * s_b


def test_sparsity_penalty_hand_example():
    # off-diagonal 0.03 < h counts, 0.2 >= h does not; the diagonal never does
    a = np.array([[0.01, 0.2], [0.03, 0.04]])
    v, g = oracle.sparsity_penalty(a, 0.1, 0.05)
    assert v == pytest.approx(0.1 * 0.03, rel=1e-15)
    np.testing.assert_array_equal(g, [[0.0, 0.0], [0.1, 0.0]])
    # the hinge is strict: an entry equal to h is not penalised
    v, g = oracle.sparsity_penalty(np.array([[0.0, 0.05], [0.0, 0.0]]), 2.0, 0.05)
    assert v == 0.0 and g[0, 1] == 0.0 and g[1, 0] == 2.0


def test_sparsity_penalty_without_hinge_is_offdiagonal_l1():
    # h above every entry: lam (sum of all entries - trace), the plain l1
    # norm of the off-diagonal part for nonnegative alpha
    rng = np.random.default_rng(3)
    a = rng.uniform(0.0, 1.0, (7, 7))
    v, g = oracle.sparsity_penalty(a, 0.3, 2.0)
    assert v == pytest.approx(0.3 * (a.sum() - np.trace(a)), rel=1e-13)
    np.testing.assert_array_equal(g, 0.3 * (1.0 - np.eye(7)))
    assert oracle.sparsity_penalty(a, 0.0, 2.0)[0] == 0.0


def test_sparsity_penalty_gradient_matches_differences():
    # away from the hinge the penalty is linear in each entry
    rng = np.random.default_rng(4)
    a = rng.uniform(0.0, 0.2, (5, 5))
    lam, h = 0.7, 0.1
    v0, g = oracle.sparsity_penalty(a, lam, h)
    eps = 1e-6
    for p in range(5):
        for q in range(5):
            if abs(a[p, q] - h) < 10 * eps:
                continue
            b = a.copy()
            b[p, q] += eps
            d = (oracle.sparsity_penalty(b, lam, h)[0] - v0) / eps
            assert d == pytest.approx(g[p, q], abs=1e-7)
