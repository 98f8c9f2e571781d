"""Pins for the oracle's inference layer (Sec. 3.5): the counter-based SplitMix64 stream, the
AIES stretch move and the Nelder-Mead simplex, checked against published generator outputs,
the stretch density, a Gaussian target's moments, exact affine invariance and hand-computed
simplex steps."""
import numpy as np
from scipy import stats

from oracle import sampler as smp


def test_splitmix64_published_outputs():
    """The first outputs of SplitMix64 seeded with 0 (the generator's published test values)."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    got = [int(v) for v in smp.splitmix64(0, np.arange(4))]
    assert got == want


def test_uniforms_are_uniform_and_independent():
    u = smp.uniform(2609, np.arange(200000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.01
    u2 = smp.uniform(2610, np.arange(200000))            # another seed: another stream
    assert abs(np.corrcoef(u, u2)[0, 1]) < 0.01


def test_stretch_factor_density():
    """z = ((a - 1) u + 1)^2 / a has the density ~ 1/sqrt(z) on [1/a, a]: its CDF is
    (sqrt(a z) - 1) / (a - 1)."""
    a = 2.0
    u = smp.uniform(7, np.arange(100000))
    z = ((a - 1) * u + 1) ** 2 / a
    cdf = lambda v: np.clip((np.sqrt(a * v) - 1) / (a - 1), 0, 1)
    assert stats.kstest(z, cdf).pvalue > 1e-3
    assert z.min() >= 1 / a and z.max() <= a


def _gauss(mu, cov):
    P = np.linalg.inv(cov)
    return lambda X: -0.5 * np.einsum("ni,ij,nj->n", X - mu, P, X - mu)


def test_aies_samples_a_correlated_gaussian():
    mu = np.array([1.0, -2.0])
    cov = np.array([[1.0, 0.8], [0.8, 2.0]])
    lp = _gauss(mu, cov)
    K = 64
    X0 = mu + 0.1 * np.random.default_rng(1).normal(size=(K, 2))
    X, l, acc, chain, _ = smp.aies(lp, X0, lp(X0), 2.0, 11, 0, 3000)
    s = chain[500:].reshape(-1, 2)
    assert np.all(np.abs(s.mean(0) - mu) < 0.1 * np.sqrt(np.diag(cov)))
    assert np.allclose(np.cov(s.T), cov, rtol=0.12, atol=0.08)
    rate = acc.sum() / (K * 3000)
    assert 0.3 < rate < 0.9


def test_aies_is_affine_invariant():
    """With the same random numbers, walkers of the target p(A^-1 (x - b)) started at A X0 + b
    follow A X + b exactly (up to rounding) and accept the same proposals."""
    mu = np.array([0.5, 1.0, -1.0])
    cov = np.diag([1.0, 0.5, 2.0])
    lp = _gauss(mu, cov)
    A = np.array([[2.0, 0.3, 0.0], [-0.5, 1.0, 0.2], [0.1, 0.0, 3.0]])
    b = np.array([10.0, -5.0, 1.0])
    Ai = np.linalg.inv(A)
    lp2 = lambda Y: lp((Y - b) @ Ai.T)
    X0 = mu + np.random.default_rng(3).normal(size=(20, 3))
    X, l, acc, ch, _ = smp.aies(lp, X0, lp(X0), 2.0, 5, 0, 200)
    Y0 = X0 @ A.T + b
    Y, l2, acc2, ch2, _ = smp.aies(lp2, Y0, lp2(Y0), 2.0, 5, 0, 200)
    assert np.array_equal(acc, acc2)
    assert np.allclose(ch2, ch @ A.T + b, rtol=1e-9, atol=1e-9)


def test_aies_rejects_outside_support_and_counts_steps():
    """log p = -inf outside a box: no walker ever leaves it; a step moves each walker at most
    once; the chain records every step."""
    lp = lambda X: np.where(np.all(np.abs(X) <= 1.0, axis=1), 0.0, -np.inf)
    X0 = np.random.default_rng(4).uniform(-0.5, 0.5, (16, 2))
    X, l, acc, ch, lc = smp.aies(lp, X0, lp(X0), 2.0, 9, 3, 100)
    assert np.all(np.abs(ch) <= 1.0)
    assert ch.shape == (100, 16, 2) and lc.shape == (100, 16)
    assert np.all(acc <= 100) and acc.sum() > 0


def test_nelder_mead_first_steps_by_hand():
    """f = x^2 + y^2 from the simplex {(0,0), (1,0), (0,1)} (all values exact in binary):
    round 1 reflects to (1,-1) (f = 2 >= f_worst) and contracts inside to (0.25, 0.5);
    round 2 reflects to (-0.75, 0.5), contracts outside to (-0.3125, 0.375)."""
    f = lambda P: np.sum(np.atleast_2d(P) ** 2, axis=1)
    S0 = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    x, v = smp.nelder_mead(f, S0, 2)
    assert np.array_equal(x[0], [[0.0, 0.0], [0.25, 0.5], [1.0, 0.0]])
    assert np.array_equal(v[0], [0.0, 0.3125, 1.0])
    x, v = smp.nelder_mead(f, S0, 4)
    assert np.array_equal(x[0], [[0.0, 0.0], [-0.3125, 0.375], [0.25, 0.5]])
    assert np.array_equal(v[0], [0.0, 0.23828125, 0.3125])


def test_nelder_mead_converges():
    quad = lambda P: (P[:, 0] - 1.0) ** 2 + 10.0 * (P[:, 1] + 2.0) ** 2
    S0 = np.array([[[3.0, 3.0], [4.0, 3.0], [3.0, 4.5]], [[-5.0, 0.0], [-4.0, 1.0], [-6.0, 2.0]]])
    x, v = smp.nelder_mead(quad, S0, 300)
    assert np.all(np.abs(x[:, 0] - [1.0, -2.0]) < 1e-6)
    rosen = lambda P: (1 - P[:, 0]) ** 2 + 100 * (P[:, 1] - P[:, 0] ** 2) ** 2
    x, v = smp.nelder_mead(rosen, np.array([[[-1.2, 1.0], [-1.0, 1.0], [-1.2, 1.2]]]), 600)
    assert np.all(np.abs(x[0, 0] - [1.0, 1.0]) < 1e-4)


def test_nelder_mead_is_affine_invariant():
    f = lambda P: (P[:, 0] - 1.0) ** 2 + 3.0 * (P[:, 1] - P[:, 0]) ** 2 + 0.5 * P[:, 2] ** 2
    A = np.array([[1.5, 0.2, 0.0], [0.0, 0.7, -0.3], [0.4, 0.0, 2.0]])
    b = np.array([1.0, 2.0, -3.0])
    Ai = np.linalg.inv(A)
    g = lambda Y: f((Y - b) @ Ai.T)
    S0 = np.random.default_rng(8).normal(size=(4, 4, 3))
    x, v = smp.nelder_mead(f, S0, 60)
    y, w = smp.nelder_mead(g, S0 @ A.T + b, 60)
    assert np.allclose(y, x @ A.T + b, rtol=1e-9, atol=1e-9)
    assert np.allclose(v, w, rtol=1e-9, atol=1e-12)


def test_nelder_mead_respects_the_prior_box():
    """f = +inf outside the box: a run started inside stays inside; its best point is the
    constrained minimum when the free minimum lies outside."""
    f0 = lambda P: (P[:, 0] - 3.0) ** 2 + (P[:, 1] - 0.5) ** 2
    f = lambda P: np.where(np.all((P >= 0) & (P <= 1), axis=1), f0(P), np.inf)
    x, v = smp.nelder_mead(f, np.array([[[0.2, 0.2], [0.4, 0.2], [0.2, 0.4]]]), 400)
    assert np.all((x >= 0) & (x <= 1))
    assert abs(x[0, 0, 0] - 1.0) < 1e-4 and abs(x[0, 0, 1] - 0.5) < 1e-3


def test_lens_likelihood_wrapper(orc):
    """chi^2 of each row inside the prior box equals the oracle's chi^2; +inf outside the box
    and for an invalid model (axis ratio above 1)."""
    from tests import lensdata
    model, truth, cons = lensdata.small_constraints(41)
    lo, hi = truth - np.abs(truth) * 0.5 - 1.0, truth + np.abs(truth) * 0.5 + 1.0
    f = smp.lens_chi2(model, cons, lo, hi)
    P = np.repeat(truth[None], 4, 0)
    P[1, 0] += 0.05
    P[2, 0] = hi[0] + 1.0                       # outside the box
    P[3, 3] = 1.2                               # q > 1 (inside a widened box)
    f2 = smp.lens_chi2(model, cons, lo - 5.0, hi + 5.0)
    v, v2 = f(P), f2(P)
    ref = orc.chi2_batch(orc.expand_batch(model, P[:2]), cons)["chi2_src"]
    assert np.array_equal(v[:2], ref)
    assert np.isinf(v[2]) and np.isinf(v2[3])
    assert np.allclose(smp.lens_logp(model, cons, lo, hi)(P[:2]), -0.5 * ref)
