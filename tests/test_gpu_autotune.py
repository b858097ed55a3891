"""The autotuner and its cache (dg2_autotune, dg2_batch_autotune, JSON tune
cache keyed by GPU architecture, precision, variant, flux, kernel form and
size class).

* a context tunes rows per wavefront x wavefronts per workgroup and stores
  the choice; a second context with the same key takes it from the cache
  without timing, and its states are bitwise those of an untuned context
  (the launch shape never changes results);
* a batch tunes rows x waves x graph length, stores it, and a second batch
  of the same members takes it from the cache; batched results stay bitwise
  those of the members stepped alone;
* an entry for another key is not used.
"""
import json

import numpy as np
import pytest

from paper_2010_02003_amd import dg2
from paper_2010_02003_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_context_autotune_is_cached_and_reused(tmp_path, precision):
    cache = str(tmp_path / "tune.json")
    sc = WL.dambreak_bump(nx=200, ny=150, precision=precision, steps=40)
    a = dg2.sim_from_scenario(sc)
    a.set_tune_cache(cache)
    rows = a.autotune(500.0)
    ra, wa, fa = a.get_launch()
    entries = json.load(open(cache))
    _say("%s: tuned rows %d waves %d; cache %s" % (precision, ra, wa, entries))
    assert rows == ra and not fa and len(entries) == 1
    key = next(iter(entries))
    assert key.startswith("gfx") and ("fp32" if precision == "fp32" else "fp64") in key and "256x256" in key
    assert entries[key]["rows"] == ra and entries[key]["waves"] == wa
    # a second context with the same key takes the shape from the cache
    b = dg2.sim_from_scenario(sc)
    b.set_tune_cache(cache)
    assert b.autotune(500.0) == ra
    assert b.get_launch() == (ra, wa, True)
    # tuned, cached and untuned runs give the same states bit for bit
    c = dg2.sim_from_scenario(sc)
    for s in (a, b, c):
        s.step(sc.steps)
    sa, sb, sc_ = (s.get_state()[0] for s in (a, b, c))
    assert np.array_equal(sa, sc_) and np.array_equal(sb, sc_)
    # another key (a different size class) is tuned afresh and added
    d = dg2.sim_from_scenario(WL.dambreak_bump(nx=100, ny=60, precision=precision))
    d.set_tune_cache(cache)
    d.autotune(300.0)
    assert not d.get_launch()[2] and len(json.load(open(cache))) == 2
    for s in (a, b, c, d):
        s.close()


def test_batch_autotune_is_cached_and_reused(tmp_path):
    cache = str(tmp_path / "tune.json")
    scs = []
    for m in range(6):
        sc = WL.ensemble_member(m)
        scs.append(sc)
    sims = [dg2.sim_from_scenario(sc) for sc in scs]
    for s in sims:
        s.step(30)  # water in the domain before tuning
    b = dg2.Batch(sims)
    b.set_tune_cache(cache)
    b.autotune(400.0)
    rows, waves, gsteps, cached = b.get_launch()
    entries = json.load(open(cache))
    _say("batch tuned: rows %d waves %d graph %d; cache %s" % (rows, waves, gsteps, entries))
    assert not cached and len(entries) == 1 and "batch" in next(iter(entries))
    b.step(40)
    b.sync()
    got = [s.get_state()[0] for s in sims]
    b.close()
    # the same members (fresh) in a second batch: shape from the cache
    sims2 = [dg2.sim_from_scenario(sc) for sc in scs]
    for s in sims2:
        s.step(30)
    b2 = dg2.Batch(sims2)
    b2.set_tune_cache(cache)
    b2.autotune(400.0)
    assert b2.get_launch() == (rows, waves, gsteps, True)
    b2.step(40)
    b2.sync()
    # and each member stepped alone
    alone = [dg2.sim_from_scenario(sc) for sc in scs]
    for s in alone:
        s.step(70)
    for g, s2, s1 in zip(got, sims2, alone):
        st1 = s1.get_state()[0]
        assert np.array_equal(g, st1) and np.array_equal(s2.get_state()[0], st1)
    b2.close()
    for s in sims + sims2 + alone:
        s.close()
