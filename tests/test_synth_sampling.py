"""The Cauchy q sampler used for importance sampling of the rates (Sec. 4.3).

It only draws inputs (points and their weights), so it is pinned against
closed forms of the wrapped Cauchy distribution rather than against the oracle:
the density's image sum, its normalisation, the distribution of the samples,
and unbiased weighted averages of functions with known zone integrals.
"""
import numpy as np
import pytest

import synth


def _density(x, gamma):
    s, c = np.sinh(2 * np.pi * gamma), np.cosh(2 * np.pi * gamma)
    return s / (c - np.cos(2 * np.pi * x))


@pytest.mark.parametrize("gamma", [0.02, 0.1, 0.5])
def test_wrapped_density_is_the_image_sum(gamma):
    # wrapping a Cauchy variable onto the unit cell sums its density over images
    x = np.linspace(-0.5, 0.5, 41)
    n = np.arange(-200000, 200001)[:, None]
    img = (gamma / np.pi / ((x[None, :] + n) ** 2 + gamma ** 2)).sum(axis=0)
    tail = 2 * gamma / np.pi / 200000.5          # both tails beyond |n| > N, to O(N^-2)
    assert np.allclose(img + tail, _density(x, gamma), rtol=1e-7)
    xs = np.linspace(-0.5, 0.5, 200001)
    assert abs(np.trapezoid(_density(xs, gamma), xs) - 1.0) < 1e-8


def test_samples_follow_the_density():
    gamma, n = 0.05, 100000
    q, w = synth.cauchy_points(11, n, gamma)
    assert q.shape == (n, 3) and w.shape == (n,)
    assert np.all(q >= -0.5) and np.all(q < 0.5)
    xs = np.linspace(-0.5, 0.5, 400001)
    p = _density(xs, gamma)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * np.diff(xs))])
    for a in range(3):
        s = np.sort(q[:, a])
        emp = np.arange(1, n + 1) / n
        ks = np.max(np.abs(np.interp(s, xs, cdf) - emp))
        assert ks < 1.63 / np.sqrt(n)             # Kolmogorov 99% point
    # the weights are 1/(n p(q)) with p the product density
    assert np.allclose(w, 1.0 / (n * np.prod(_density(q, gamma), axis=1)))


def test_weighted_averages_are_unbiased():
    # zone averages of 1, cos^2(2 pi x) cos^2(2 pi y), and exp(-|q|^2/s^2)
    # (a peak at Gamma, integral by the product of error functions)
    from math import erf, pi, sqrt
    s = 0.08
    exact_peak = (s * sqrt(pi) * erf(0.5 / s)) ** 3
    for gamma in (0.03, 0.2):
        q, w = synth.cauchy_points(23, 200000, gamma)
        for f, exact in ((np.ones(len(q)), 1.0),
                         (np.cos(2 * np.pi * q[:, 0]) ** 2 * np.cos(2 * np.pi * q[:, 1]) ** 2, 0.25),
                         (np.exp(-(q ** 2).sum(axis=1) / s ** 2), exact_peak)):
            terms = len(q) * w * f
            est, se = terms.mean(), terms.std() / np.sqrt(len(q))
            assert abs(est - exact) <= 5 * se, (gamma, est, exact, se)


def test_cauchy_reduces_variance_for_a_peak_at_gamma():
    s = 0.04
    f = lambda q: np.exp(-(q ** 2).sum(axis=1) / s ** 2)
    qc, wc = synth.cauchy_points(5, 50000, 0.04)
    qu = synth.random_points(5, 50000)
    qu = qu - np.floor(qu + 0.5)                  # same cell as the Cauchy points
    var_c = np.var(len(qc) * wc * f(qc))
    var_u = np.var(f(qu))
    from math import erf, pi, sqrt
    exact = (s * sqrt(pi) * erf(0.5 / s)) ** 3
    assert abs(f(qu).mean() - exact) <= 5 * np.sqrt(var_u / len(qu))
    assert abs(np.mean(len(qc) * wc * f(qc)) - exact) <= 5 * np.sqrt(var_c / len(qc))
    assert var_c < 0.01 * var_u


# --------------------------------------------------------------- counter-based draws

def test_philox_known_answers():
    """Philox4x32-10 against the known-answer vectors of its authors' reference
    implementation (counter, key -> output)."""
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, want in cases:
        got = synth.philox4x32_10(*[np.uint32(x) for x in ctr], np.uint32(key[0]), np.uint32(key[1]))
        assert tuple(int(x) for x in got) == want


def test_counter_normals_moments_and_entry_access():
    """The Irwin-Hall(12) variates have mean 0 and variance 1 (sample of 2e5),
    lie in [-6, 6], and an entry drawn alone equals the same entry of the whole
    tensor (the draw depends only on the entry's index)."""
    t = np.arange(200_000)
    xr, xi = synth.counter_normals(t, 1234567)
    for x in (xr, xi):
        assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
        assert x.min() >= -6.0 and x.max() <= 6.0
    assert abs(np.corrcoef(xr, xi)[0, 1]) < 0.01
    env = np.abs(np.random.default_rng(3).random((5, 7))) + 0.1
    full = synth.counter_coupling(env, 12, 99)
    idx = np.array([0, 1, 11, 12, 419])
    part = synth.counter_coupling(env, 12, 99, entries=idx)
    assert np.array_equal(full.reshape(-1)[idx], part)
