"""Multi-index Monte Carlo with sample reuse: the reference estimator pinned
to closed forms (unbiasedness by exact enumeration, the sampler's tail law,
Theorem 1 by direct cost accounting), the product's host arithmetic against
it, and on the GPU the batched estimator against the reference estimator fed
with oracle solutions of the same samples."""
import itertools
import math

import numpy as np
import pytest

from oracle import mimc_oracle as MO
from oracle import normals as NR
from paper_1907_12334_amd import inputs as I
from paper_1907_12334_amd import mimc as M


def test_unbiased_by_exact_enumeration():
    """E[Y] over the geometric index equals the telescoped sum of the
    differences, here a closed form (no truncation of the index set)."""
    r = (0.9, 1.3)
    dq = {(a, b): 0.3 * 2.0 ** (-2 * a) * 3.0 ** (-b) for a in range(80) for b in range(80)}
    total = 0.3 / ((1 - 1 / 4) * (1 - 1 / 3))
    ey = 0.0
    for L1, L2 in itertools.product(range(45), range(45)):
        prob = ((1 - math.exp(-r[0])) * math.exp(-r[0] * L1)) * ((1 - math.exp(-r[1])) * math.exp(-r[1] * L2))
        ey += prob * MO.sample_y(dq, (L1, L2), r)
    assert abs(ey - total) <= 1e-10 * total


def test_geometric_sampler_tail_law():
    """P(L >= l) = exp(-r l): exact at the inverse-transform boundaries, and
    empirically on many draws."""
    r = 1.7
    for l in range(6):
        u = math.exp(-r * l)
        assert MO.draw_index((r,), (u,))[0] == l
        assert MO.draw_index((r,), (u * (1 + 1e-12),))[0] == l - 1 if l > 0 else True
    u = I.mimc_uniforms(200000, 0)[:, 0]
    L = np.array([MO.draw_index((r,), (x,))[0] for x in u[:20000]])
    for l in range(4):
        p = math.exp(-r * l)
        assert abs(np.mean(L >= l) - p) <= 4 * math.sqrt(p * (1 - p) / len(L)) + 1e-12


@pytest.mark.parametrize("beta,gamma", [((4.73, 4.47), (1.27, 1.21)), ((2.21, 2.57), (1.21, 1.34)),
                                        ((1.36, 1.51), (1.49, 1.26)), ((4.0, 4.0), (1.0, 1.0))])
def test_theorem1_by_direct_cost_accounting(beta, gamma):
    """Theorem 1 against the sums it summarises: sample sizes N_tau ~
    prod 2^(-(gamma+beta) tau / 2), the reuse-reduced sizes of its proof and
    costs prod 2^(gamma tau), summed over a large box; and in two
    directions the factorised form (1 - a1)(1 - a2)."""
    K = 120
    a = [2.0 ** (-(g + b) / 2.0) for b, g in zip(beta, gamma)]
    num = den = 0.0
    for t1 in range(K):
        for t2 in range(K):
            N = lambda x, y: 2.0 ** (-(gamma[0] + beta[0]) * x / 2) * 2.0 ** (-(gamma[1] + beta[1]) * y / 2)
            C = 2.0 ** (gamma[0] * t1) * 2.0 ** (gamma[1] * t2)
            Nr = N(t1, t2) - (N(t1 + 1, t2) + N(t1, t2 + 1) - N(t1 + 1, t2 + 1))
            num += Nr * C
            den += N(t1, t2) * C
    ratio = MO.cost_ratio(beta, gamma)
    assert abs(ratio - num / den) <= 1e-12
    assert abs(ratio - (1 - a[0]) * (1 - a[1])) <= 1e-14


def test_estimate_matches_sample_statistics():
    ys = list(np.random.default_rng(3).standard_normal(50))
    e, v = MO.estimate(ys)
    assert abs(e - np.mean(ys)) <= 1e-15 and abs(v - np.var(ys, ddof=1) / len(ys)) <= 1e-15


def test_product_host_arithmetic_matches_reference():
    """The driver's vectorised draws, weights and statistics equal the
    reference's loops on the same uniforms."""
    r = M.initial_rates()
    u = I.mimc_uniforms(500, 3)
    L = M.draw_indices(u, r, lmax=30)
    ref = np.array([MO.draw_index(tuple(r), tuple(x)) for x in u])
    assert np.array_equal(L, ref)
    rng = np.random.default_rng(9)
    for P, Q in [(0, 0), (3, 2), (1, 5)]:
        d = rng.standard_normal((P + 1) * (Q + 1))
        table = {(a, b): d[a * (Q + 1) + b] for a in range(P + 1) for b in range(Q + 1)}
        assert abs(np.dot(d, M.reuse_weights(P, Q, r)) - MO.sample_y(table, (P, Q), tuple(r))) <= 1e-12 * (
            1 + abs(MO.sample_y(table, (P, Q), tuple(r))))
    assert abs(M.initial_rates()[0] - math.log(2) * 5 / 2) <= 1e-15


class _FakeSolves(M.MSGMIMC):
    """The estimator's host logic with solves replaced by given per-grid
    differences, statuses and cycle counts (no GPU)."""

    def __init__(self, make, **kw):
        super().__init__(handle=None, **kw)
        self.make = make

    def solve_batch(self, L):
        ids = np.arange(self.next_sample_id, self.next_sample_id + len(L))
        self.next_sample_id += len(L)
        out = [self.make(int(i), int(P), int(Q)) for i, (P, Q) in zip(ids, L)]
        return [o[0] for o in out], np.array([o[1] for o in out]), [o[2] for o in out], ids


@pytest.mark.parametrize("bad", ["maxiter", "nonfinite", "nan_difference"])
def test_failed_samples_stop_the_estimator(bad):
    """A sample that hit the cycle cap, went non-finite, or returned a NaN
    difference raises MIMCFailure naming it, and its batch adds nothing."""
    def make(i, P, Q):
        n = (P + 1) * (Q + 1)
        d, st = np.full(n, 1e-3), 0
        if i == 5:
            st = {"maxiter": 1, "nonfinite": 2, "nan_difference": 0}[bad]
            if bad != "maxiter":
                d[-1] = np.nan
        return d, st, np.full(n, 3, dtype=np.int32)
    est = _FakeSolves(make, lmax=3, r0=np.array([0.7, 0.7]), learn=False)
    with pytest.raises(M.MIMCFailure) as err:
        est.add_batch(16)
    assert err.value.failed[0][0] == 5 and len(est.ys) == 0 and est.batches == 0


def test_work_rates_are_fitted_from_the_cycle_counts():
    """With the same cycle count on every grid, the work of a sample at L is
    sum_tau (tau1+1)(tau2+1) c^2 2^(tau1+tau2); the fitted gamma follows the
    growth of that sum (between 1 and 2 per direction over small indices)
    and changes when the cycle counts grow with the index."""
    def flat(i, P, Q):
        n = (P + 1) * (Q + 1)
        return np.full(n, 2.0 ** -(P + Q)), 0, np.full(n, 4, dtype=np.int32)
    est = _FakeSolves(flat, lmax=4, r0=np.array([0.4, 0.4]), learn=True)
    for _ in range(6):
        est.add_batch(256)
    g1 = est.gamma.copy()
    assert np.all(g1 > 1.0) and np.all(g1 < 2.0)
    assert abs(M.sample_work(4, 1, 0, np.array([2, 3])) - (2 * 16 + 3 * 2 * 32)) < 1e-12

    def growing(i, P, Q):
        n = (P + 1) * (Q + 1)
        cyc = np.array([[4 * 2 ** a for b in range(Q + 1)] for a in range(P + 1)], dtype=np.int32).ravel()
        return np.full(n, 2.0 ** -(P + Q)), 0, cyc
    est2 = _FakeSolves(growing, lmax=4, r0=np.array([0.4, 0.4]), learn=True)
    for _ in range(6):
        est2.add_batch(256)
    assert est2.gamma[0] > g1[0] + 0.5 and abs(est2.gamma[1] - g1[1]) < 0.3


def _noisy_tables(seed, lmax):
    rng = np.random.default_rng(seed)
    t = np.arange(lmax + 1)
    V = 2.0 ** (-3.1 * t[:, None] - 1.7 * t[None, :]) * np.exp(0.8 * rng.standard_normal((lmax + 1, lmax + 1)))
    C = 2.0 ** (1.2 * t[:, None] + 1.4 * t[None, :]) * np.exp(0.3 * rng.standard_normal((lmax + 1, lmax + 1)))
    return V, C


def test_learned_pmf_is_geometric_under_product_laws():
    """With V_tau = 2^(-beta.tau) and C_tau = 2^(gamma.tau) exactly, N_tau of
    eq. Nell is prod exp(-r_j tau_j) with r_j = log(2)(beta_j + gamma_j)/2, so
    the learned tail is the geometric one (the paper's derivation of the
    geometric choice), whatever the mixing weight."""
    beta, gamma, lmax = (3.3, 2.1), (1.3, 1.1), 6
    r = [math.log(2) * (b + g) / 2 for b, g in zip(beta, gamma)]
    V = {(a, b): 2.0 ** (-beta[0] * a - beta[1] * b) for a in range(lmax + 1) for b in range(lmax + 1)}
    C = {(a, b): 2.0 ** (gamma[0] * a + gamma[1] * b) for a in range(lmax + 1) for b in range(lmax + 1)}
    for eps in (0.0, 0.3):
        pi, p = MO.learned_distribution(V, C, (0.5, 0.5) if eps == 0 else r, lmax, eps)
        for k, x in MO.geometric_tail(r, lmax).items():
            assert abs(p[k] - x) <= 1e-13
        assert abs(pi[(0, 0)] - (1 - math.exp(-r[0])) * (1 - math.exp(-r[1]))) <= 1e-13
        # capped at the box edge: P(L = (lmax, 0)) holds the mass beyond it
        assert abs(pi[(lmax, 0)] - math.exp(-r[0] * lmax) * (1 - math.exp(-r[1]))) <= 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_learned_pmf_is_a_distribution_with_its_own_tail(seed):
    """On noisy tables (tails that are not those of any distribution): the
    pmf is non-negative and sums to one, every index of the box has positive
    probability (the geometric floor), p_0 = 1, p decreases in each
    direction, and p is the tail of pi (inclusion-exclusion gives pi back)."""
    lmax = 5
    Va, Ca = _noisy_tables(seed, lmax)
    V = {(a, b): Va[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    C = {(a, b): Ca[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    raw = MO.pmf_from_tail(MO.empirical_tail(V, C, lmax), lmax)
    assert min(raw.values()) < 0           # the case the clipping is for
    pi, p = MO.learned_distribution(V, C, (1.0, 1.0), lmax, 0.1)
    assert min(pi.values()) > 0 and abs(sum(pi.values()) - 1) <= 1e-14
    assert abs(p[(0, 0)] - 1) <= 1e-14
    for (a, b), x in p.items():
        if a > 0:
            assert x <= p[(a - 1, b)] + 1e-15
        if b > 0:
            assert x <= p[(a, b - 1)] + 1e-15
    back = MO.pmf_from_tail(p, lmax)
    assert max(abs(back[k] - pi[k]) for k in pi) <= 1e-14


def test_learned_pmf_unbiased_by_exact_enumeration():
    """E[Y] = sum over L of pi(L) Y(L) equals the sum of the differences over
    the box, for any valid pmf and its tail (the telescoping identity)."""
    lmax = 5
    Va, Ca = _noisy_tables(7, lmax)
    V = {(a, b): Va[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    C = {(a, b): Ca[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    pi, p = MO.learned_distribution(V, C, (0.8, 1.9), lmax, 0.05)
    rng = np.random.default_rng(4)
    dq = {k: float(rng.standard_normal()) for k in pi}
    ey = sum(pi[L] * MO.sample_y_tail(dq, L, p) for L in pi)
    assert abs(ey - sum(dq.values())) <= 1e-12 * (1 + sum(abs(x) for x in dq.values()))


def test_learned_pmf_host_arithmetic_matches_reference():
    """The driver's vectorised pmf, tail and draws equal the reference's loops."""
    lmax = 6
    Va, Ca = _noisy_tables(11, lmax)
    V = {(a, b): Va[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    C = {(a, b): Ca[a, b] for a in range(lmax + 1) for b in range(lmax + 1)}
    r = np.array([1.1, 0.7])
    pi_ref, p_ref = MO.learned_distribution(V, C, tuple(r), lmax, 0.1)
    pi, p = M.learned_distribution(Va, Ca, r, 0.1)
    for (a, b) in pi_ref:
        assert abs(pi[a, b] - pi_ref[(a, b)]) <= 1e-15 and abs(p[a, b] - p_ref[(a, b)]) <= 1e-14
    u = I.mimc_uniforms(3000, 5)[:, 0]
    L = M.draw_indices_pmf(u, pi)
    ref = np.array([MO.draw_index_pmf(pi_ref, lmax, float(x)) for x in u])
    assert np.array_equal(L, ref)


def test_learned_pmf_estimator_is_unbiased_with_fake_solves():
    """The estimator with the learned pmf on fake solves whose differences
    have known means (2^-(2a+b) times a unit-mean normal factor): the learned
    distribution leaves the geometric one, and the estimate is within four
    RMSE of the exact sum over the box."""
    lmax = 5

    def make(i, P, Q):
        rng = np.random.default_rng(1000 + i)
        n = (P + 1) * (Q + 1)
        a = np.repeat(np.arange(P + 1), Q + 1)
        b = np.tile(np.arange(Q + 1), P + 1)
        d = 2.0 ** -(2 * a + b) * (1 + rng.standard_normal(n))
        return d, 0, np.full(n, 4, dtype=np.int32)
    est = _FakeSolves(make, lmax=lmax, r0=np.array([0.5, 0.5]), learn=True, pmf="learned")
    res = est.run(tol=3e-2, batch=512)
    exact = sum(2.0 ** -(2 * a + b) for a in range(lmax + 1) for b in range(lmax + 1))
    assert res.pmf == "learned" and abs(res.E - exact) <= 4 * res.rmse
    assert np.max(np.abs(est.tail - M.geometric_tail(est.r, lmax))) > 1e-3
    assert abs(est.pi.sum() - 1) <= 1e-12 and est.pi.min() > 0


def test_running_statistics_match_direct_ones():
    """Per-index variances merged batch by batch, and E and V of the Y's,
    equal the direct sample statistics of every value seen."""
    seen = {}

    def make(i, P, Q):
        rng = np.random.default_rng(i)
        n = (P + 1) * (Q + 1)
        d = 3.0 + rng.standard_normal(n) * 0.1
        for a in range(P + 1):
            for b in range(Q + 1):
                seen.setdefault((a, b), []).append(d[a * (Q + 1) + b])
        return d, 0, np.full(n, 2, dtype=np.int32)
    est = _FakeSolves(make, lmax=3, r0=np.array([0.6, 0.9]), learn=False)
    for n in (17, 64, 5):
        est.add_batch(n)
    for k, xs in seen.items():
        if len(xs) >= 2:
            assert abs(est.variance(k, 2) - np.var(xs, ddof=1)) <= 1e-12 * np.var(xs, ddof=1)
    e, v = est.estimate()
    e_ref, v_ref = MO.estimate(est.ys)
    assert abs(e - e_ref) <= 1e-13 * abs(e_ref) and abs(v - v_ref) <= 1e-10 * v_ref


def test_pmf_option_is_checked():
    with pytest.raises(ValueError):
        _FakeSolves(lambda *a: None, pmf="uniform")


@pytest.mark.gpu
def test_batched_estimator_matches_reference_on_oracle_solutions():
    """Two batches of 24 samples, fixed rates, indices capped at 3: the GPU
    estimator's E and V equal the reference estimator's on oracle solutions
    of the same samples (same uniforms, the same normal streams) to the
    FP64 bar."""
    import torch
    from oracle import binding as O
    from paper_1907_12334_amd import msg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = msg.Handle(0)
    est = M.MSGMIMC(h, I.KL10, c=4, kind=msg.QOI_POINT, opts=msg.SolveOpts(tol=1e-10), lmax=3,
                    r0=np.array([0.6, 0.8]), learn=False)
    est.add_batch(24)
    est.add_batch(24)
    e, v = est.estimate()
    ys, sid = [], 0
    for b in range(2):
        u = I.mimc_uniforms(24, b, est.seed)
        for x in u:
            L = MO.draw_index((0.6, 0.8), tuple(x))
            L = (min(L[0], 3), min(L[1], 3))
            xi = NR.kl_normals(I.KL10.n_terms, [sid], est.seed)[0]
            sid += 1
            kx, ky = O.hierarchy_field(4, L[0], L[1], I.KL10.as_dict(), xi)
            r = O.fmsg_solve(4, L[0], L[1], kx, ky, O.opts(tol=1e-10))
            q = O.qoi(4, L[0], L[1], r["u"], kx, O.QOI_POINT)
            dq = O.delta_q(L[0], L[1], q)
            table = {(a, c): dq[a * (L[1] + 1) + c] for a in range(L[0] + 1) for c in range(L[1] + 1)}
            ys.append(MO.sample_y(table, L, (0.6, 0.8)))
    e0, v0 = MO.estimate(ys)
    assert abs(e - e0) <= 1e-9 * abs(e0) and abs(v - v0) <= 1e-7 * v0
    assert len(est.counts) > 3                        # the draws spread over several rectangles


def test_matern_prior_hyperparameters_span_the_paper_ranges():
    """Section 5's hyperparameters: eta uniform on [1/16, 1/4], theta uniform
    on [-30, 30] degrees, mapped affinely from the uniforms."""
    pr = I.MATERN_PAPER
    assert (pr.lam, pr.nu, pr.pad) == (0.25, 0.5, 0)
    eta, theta = pr.hyperparameters(np.array([[1.0, 1.0], [0.5, 0.5], [1e-12, 1e-12]]))
    assert np.allclose(eta, [0.25, 0.15625, 1 / 16]) and np.allclose(np.degrees(theta), [30.0, 0.0, -30.0])
    eta, theta = pr.hyperparameters(I.mimc_uniforms(20000, 0, 99))
    assert eta.min() >= 1 / 16 and eta.max() <= 0.25 and abs(eta.mean() - 0.15625) < 2e-3
    assert abs(np.degrees(theta)).max() <= 30.0 and abs(np.degrees(theta).mean()) < 0.5


@pytest.mark.gpu
def test_matern_prior_estimator_matches_reference_on_oracle_solutions():
    """The paper's field model inside the estimator: every sample draws eta
    and theta, its Matern field comes from the device sampler and its solve
    from full MSG.  Two batches of 16 samples, fixed rates, indices capped at
    2: E and V equal the reference estimator's on oracle fields and oracle
    solutions of the same samples (same uniforms, same Philox stream)."""
    import torch
    from oracle import binding as O
    from oracle import matern_oracle as MT
    from paper_1907_12334_amd import msg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = msg.Handle(0)
    r = (0.6, 0.8)
    est = M.MSGMIMC(h, c=4, kind=msg.QOI_POINT, opts=msg.SolveOpts(tol=1e-10), lmax=2, r0=np.array(r),
                    learn=False, prior=I.MATERN_PAPER)
    print("matern mimc: 2 batches of 16", flush=True)
    est.add_batch(16)
    est.add_batch(16)
    e, v = est.estimate()
    ys, sid = [], 0
    for b in range(2):
        u = I.mimc_uniforms(16, b, est.seed)
        uh = I.mimc_uniforms(16, b, est.seed + 1)
        for x, (ue, ut) in zip(u, uh):
            L = MO.draw_index(r, tuple(x))
            L = (min(L[0], 2), min(L[1], 2))
            eta, theta = 1 / 16 + (1 / 4 - 1 / 16) * ue, math.radians(-30 + 60 * ut)
            kx, ky, ratio = MT.hierarchy_field(4, L[0], L[1], 0.25, 0.5, eta, theta, sid, est.seed)
            assert ratio > 0.0
            sid += 1
            res = O.fmsg_solve(4, L[0], L[1], kx, ky, O.opts(tol=1e-10))
            assert res["status"] == 0
            q = O.qoi(4, L[0], L[1], res["u"], kx, O.QOI_POINT)
            dq = O.delta_q(L[0], L[1], q)
            table = {(a, c): dq[a * (L[1] + 1) + c] for a in range(L[0] + 1) for c in range(L[1] + 1)}
            ys.append(MO.sample_y(table, L, r))
    e0, v0 = MO.estimate(ys)
    assert abs(e - e0) <= 1e-9 * abs(e0) and abs(v - v0) <= 1e-7 * v0
    assert len(est.counts) > 3 and est.min_eig_ratio > 0.0
