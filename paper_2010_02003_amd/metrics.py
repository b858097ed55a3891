"""Agreement statistics of gauge time series (Sec. 3, Eq. 13-14).

The paper compares a modelled series V^M (water level or velocity at a
sampling point) with a reference series V^R of the same length N_s through

* the R-squared coefficient, Eq. (13): the square of the correlation
  coefficient of the two series (1 for any increasing or decreasing affine
  image of the reference, 0 for an uncorrelated series);
* the L1-norm error, Eq. (14): the mean absolute difference of the two
  series over their N_s entries.

These run on the host over series read back with ``Sim.read_gauges`` (whose
samples hold h, eta, u, v per gauge: eta is the water level, hypot(u, v) the
speed) or any arrays; they post-process results and are no step of the time
integration.  Both take the series along axis 0, so an array (N_s, n_gauges)
gives one value per gauge.
"""
import numpy as np


def _pair(ref, model):
    r = np.asarray(ref, dtype=np.float64)
    m = np.asarray(model, dtype=np.float64)
    if r.shape != m.shape:
        raise ValueError("reference and model series differ in shape: %s vs %s" % (r.shape, m.shape))
    if r.shape[0] < 1:
        raise ValueError("empty time series")
    return r, m


def r_squared(ref, model):
    """Eq. (13): [sum (R - mean R)(M - mean M) / sqrt(sum (R - mean R)^2 sum (M - mean M)^2)]^2.

    NaN where either series is constant (the correlation is undefined)."""
    r, m = _pair(ref, model)
    dr = r - r.mean(axis=0)
    dm = m - m.mean(axis=0)
    num = (dr * dm).sum(axis=0)
    den = np.sqrt((dr * dr).sum(axis=0) * (dm * dm).sum(axis=0))
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), np.nan)
    return c * c


def l1_error(ref, model):
    """Eq. (14): (1/N_s) sum |R - M| over the series."""
    r, m = _pair(ref, model)
    return np.abs(r - m).mean(axis=0)

