"""Packing towers into workgroups: results do not depend on the pack size, and the pack-size
tuner picks one of its candidates and reuses a cached choice."""
import sys

import numpy as np
import pytest

from paper_2606_28394_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sorted_contacts(c):
    return c[np.lexsort((c["slot"], c["body_b"], c["body_a"]))]


def test_pack_size_does_not_change_results(J):
    """A tower's contacts, colours and sweeps involve its own bodies only, so the same batch
    packed one tower per workgroup, at the library's size and many towers per workgroup steps
    to the same bits (the same kernel instantiation runs all three)."""
    sc = W.tilted_towers(3, 40, seed=11, n_steps=30)
    ref = None
    for pb in (0, 40, 250):
        _say(f"pack_bodies {pb}: 40 tilted towers, 30 steps")
        w = J.World(sc, pack_bodies=pb)
        w.step(30)
        st = w.state()
        s = w.stats()
        assert s.error_word == 0
        cnt = [int(w.stats(t).manifolds) for t in range(sc["n_towers"])]
        con = [_sorted_contacts(w.contacts(t)) for t in (0, 17, 39)]
        w.close()
        if ref is None:
            ref = (st, cnt, con)
            continue
        for a, b in zip(ref[0], st):
            assert np.array_equal(a, b), f"pack_bodies {pb}: state differs from the library's packing"
        assert cnt == ref[1]
        for a, b in zip(ref[2], con):
            assert len(a) == len(b)
            for f in ("body_a", "body_b", "slot", "colour", "point", "normal", "depth", "lambda_n", "lambda_t1",
                      "lambda_t2"):
                assert np.array_equal(a[f], b[f]), f"pack_bodies {pb}: contact field {f} differs"


def test_tuner_picks_a_candidate_and_caches(J, tmp_path):
    from paper_2606_28394_amd import autotune as A
    sc = W.tilted_towers(3, 64, seed=12, n_steps=10)
    cache = str(tmp_path / "tune.json")
    _say("tuner: 64 tilted towers, candidates 0 and 40")
    r = A.tune_pack_bodies(sc, candidates=(0, 40), steps=4, lead_in=4, cache=cache, log=_say)
    assert r["pack_bodies"] in (0, 40) and not r["cached"]
    assert all(v > 0 for v in r["tower_steps_per_s"].values())
    again = A.tune_pack_bodies(sc, candidates=(0, 40), steps=4, lead_in=4, cache=cache)
    assert again["cached"] and again["pack_bodies"] == r["pack_bodies"]
    other = A.tune_pack_bodies(sc, candidates=(0, 40), steps=5, lead_in=4, cache=cache)
    assert not other["cached"]


def _run(J, sc, steps, chunks=1, episodes=False, **kw):
    w = J.World(sc, **kw)
    if episodes:
        w.begin_episodes()
    for _ in range(chunks):
        w.step(steps // chunks)
    out = (w.state(), [_sorted_contacts(w.contacts(t)) for t in range(sc["n_towers"])], w.stats(),
           [w.episode(t) for t in range(sc["n_towers"])] if episodes else None)
    w.close()
    return out


@pytest.mark.parametrize("case", ["removal", "removal_warm", "tilted_variants", "tilted_cone", "episodes"])
def test_small_batch_workgroups_match_one_wave(J, case):
    """A small batch steps one tower per four-wave workgroup whose lane pairs keep their manifold's
    row terms in registers through the sweeps; the same batch with small_batch = -1 runs one wave
    per tower.  Both must give the same bits: states, contacts, counters (and episode records)."""
    kw, episodes, steps = {}, False, 120
    if case.startswith("removal") or case == "episodes":
        full = W.cfg2(0, n_steps=600)
        sc = W.subset(full, [mu * 150 + i for mu in range(3) for i in range(8)])
        steps = 400 if case == "episodes" else 240
        if case == "removal_warm":
            kw["warm_start"] = 1
        episodes = case == "episodes"
    else:
        sc = W.tilted_towers(5, 24, levels_range=(8, 24), n_steps=steps)
        extra = dict(restitution_bias=1, manifold_mode=1) if case == "tilted_variants" else dict(friction_cone=1)
        sc = dict(sc, params=dict(sc["params"], **extra))
    a = _run(J, sc, steps, chunks=2, episodes=episodes, small_batch=0, **kw)
    b = _run(J, sc, steps, chunks=2, episodes=episodes, small_batch=-1, **kw)
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    for ca, cb in zip(a[1], b[1]):
        assert len(ca) == len(cb)
        for f in ca.dtype.names:
            assert np.array_equal(ca[f], cb[f]), f
    for f in ("candidates", "manifolds", "points", "contact_iters", "colours", "error_word"):
        assert getattr(a[2], f) == getattr(b[2], f), f
    assert a[2].residual_rms == b[2].residual_rms
    if episodes:
        for ea, eb in zip(a[3], b[3]):
            assert bytes(ea) == bytes(eb)
    _say(case, "bit for bit over", steps, "steps; manifolds", a[2].manifolds)
