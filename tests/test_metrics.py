"""Pins of the gauge statistics of Sec. 3, Eq. (13)-(14)
(paper_2010_02003_amd/metrics.py), against what their definitions fix:
R^2 is 1 for an affine image of the reference (either sign of slope), 0 for
an uncorrelated series, the squared Pearson coefficient of scipy, and
symmetric; the L1-norm error of a constant shift is that shift, and equals
a brute-force sum on small series."""
import numpy as np
import pytest
from scipy import stats

from paper_2010_02003_amd import metrics as M


def test_r_squared_of_affine_images_is_one():
    t = np.linspace(0.0, 3600.0, 241)
    ref = 1.2 + 0.4 * np.sin(t / 500.0) + 1e-4 * t
    for a, b in ((1.0, 0.0), (2.5, -3.0), (-0.7, 10.0)):
        assert M.r_squared(ref, a * ref + b) == pytest.approx(1.0, abs=1e-14)


def test_r_squared_of_uncorrelated_series_is_zero():
    t = np.arange(400) * (2.0 * np.pi / 400)
    assert abs(M.r_squared(np.sin(t), np.cos(t))) < 1e-28
    assert abs(M.r_squared(np.sin(t), np.sin(2.0 * t))) < 1e-28


def test_r_squared_matches_pearson_and_is_symmetric():
    rng = np.random.default_rng(11)
    for n in (2, 3, 17, 500):
        r = rng.normal(size=n)
        m = 0.3 * r + rng.normal(size=n)
        want = stats.pearsonr(r, m)[0] ** 2
        assert M.r_squared(r, m) == pytest.approx(want, rel=1e-12)
        assert M.r_squared(m, r) == pytest.approx(want, rel=1e-12)
        assert 0.0 <= M.r_squared(r, m) <= 1.0


def test_r_squared_per_gauge_and_constant_series():
    rng = np.random.default_rng(12)
    R = rng.normal(size=(50, 3))
    Mo = R.copy()
    Mo[:, 1] = rng.normal(size=50)
    Mo[:, 2] = 5.0  # a gauge that stays dry: correlation undefined
    r2 = M.r_squared(R, Mo)
    assert r2.shape == (3,)
    assert r2[0] == pytest.approx(1.0, abs=1e-14)
    assert r2[1] == pytest.approx(stats.pearsonr(R[:, 1], Mo[:, 1])[0] ** 2, rel=1e-12)
    assert np.isnan(r2[2])


def test_l1_error_is_the_mean_absolute_deviation():
    rng = np.random.default_rng(13)
    ref = rng.uniform(0.0, 2.0, size=37)
    assert M.l1_error(ref, ref + 0.25) == pytest.approx(0.25, abs=1e-15)
    assert M.l1_error(ref, ref - 0.25) == pytest.approx(0.25, abs=1e-15)
    mod = rng.uniform(0.0, 2.0, size=37)
    brute = 0.0
    for a, b in zip(ref, mod):
        brute += abs(a - b)
    assert M.l1_error(ref, mod) == pytest.approx(brute / 37, rel=1e-14)
    assert M.l1_error(ref, ref) == 0.0


def test_metrics_reject_mismatched_or_empty_series():
    with pytest.raises(ValueError):
        M.r_squared(np.zeros(4), np.zeros(5))
    with pytest.raises(ValueError):
        M.l1_error(np.zeros(0), np.zeros(0))
