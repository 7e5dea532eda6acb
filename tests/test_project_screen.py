"""The division-free frustum screen of the projection kernel.

The projection kernel culls a (view, Gaussian) pair without dividing when
|p_x| > fl(fl(limx * p_z) * (1 + 2^-10)) (and that threshold is above
2^-100), and decides every other pair with the exact binary32 test
|fl(p_x / p_z)| <= limx of Sec. 3.2.1's projection.  The screen must never
cull a pair that the exact test keeps, or the binning would differ from a
plain evaluation.  This checks that implication in IEEE binary32 (numpy
rounds every float32 operation to nearest) on random pairs and on pairs
placed on the threshold itself, one and a few ulps around it.
"""
import numpy as np

SLACK = np.float32(1.0 + 2.0 ** -10)
TINY = np.float32(2.0 ** -100)


def screened_out(p0, p2, lim):
    thr = (lim * p2) * SLACK  # float32 throughout
    return (np.abs(p0) > thr) & (thr > TINY)


def exact_keeps(p0, p2, lim):
    return np.abs(p0 / p2) <= lim


def _check(p0, p2, lim):
    p0, p2, lim = (np.asarray(a, dtype=np.float32) for a in (p0, p2, lim))
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        bad = screened_out(p0, p2, lim) & exact_keeps(p0, p2, lim)
    assert not bad.any(), (p0[bad][:5], p2[bad][:5], lim[bad][:5])


def test_screen_never_culls_a_kept_pair_random():
    rng = np.random.default_rng(7)
    m = 400_000
    lim = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), m)).astype(np.float32)
    p2 = np.exp(rng.uniform(np.log(1e-3), np.log(1e6), m)).astype(np.float32)
    p0 = (lim * p2 * rng.uniform(-1.01, 1.01, m)).astype(np.float32)
    _check(p0, p2, lim)


def test_screen_never_culls_a_kept_pair_at_the_threshold():
    rng = np.random.default_rng(11)
    m = 200_000
    lim = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), m)).astype(np.float32)
    p2 = np.exp(rng.uniform(np.log(0.2), np.log(1e4), m)).astype(np.float32)
    thr = (lim * p2) * SLACK
    kept_edge = (lim * p2).astype(np.float32)  # where the exact test flips
    for base in (thr, kept_edge):
        x = base.copy()
        for _ in range(4):  # the base and three ulps either side
            _check(x, p2, lim)
            _check(-x, p2, lim)
            _check(np.nextafter(base, np.float32(0)), p2, lim)
            x = np.nextafter(x, np.float32(np.inf))
            base = np.nextafter(base, np.float32(0))


def test_screen_keeps_special_values_for_the_exact_test():
    # non-finite or huge values must reach the exact test, never be screened
    p2 = np.float32([np.inf, 1.0, 1.0, 3e38])
    p0 = np.float32([1.0, np.nan, 2.0, 3e38])
    lim = np.float32([1.0, 1.0, np.inf, 1.0])
    with np.errstate(over="ignore", invalid="ignore"):
        assert not screened_out(p0, p2, lim).any()


def test_screen_culls_most_of_what_the_exact_test_culls():
    # the screen is only worth having if it rarely passes a culled pair
    rng = np.random.default_rng(3)
    m = 100_000
    lim = np.float32(1.3)
    p2 = rng.uniform(0.2, 10.0, m).astype(np.float32)
    p0 = rng.uniform(-20.0, 20.0, m).astype(np.float32)
    culled = ~exact_keeps(p0, p2, lim)
    passed_but_culled = culled & ~screened_out(p0, p2, lim)
    assert passed_but_culled.sum() <= 1e-3 * culled.sum()
