"""The C ABI's device-side error handling and zero-copy views, on the GPU.

- A tower whose state is non-finite at the start of a step is frozen: its bodies keep their
  state, the other towers of its pack step to the same bits as without it, and the next syncing
  call returns JG_ENAN once.
- Colliding pairs beyond a pack's capacity (forced from the host with a small
  manifolds_per_body) are dropped from the end of the canonical list: the kept pairs are the
  oracle's first ones, and the next syncing call returns JG_ECAPACITY once.
- Manifolds beyond 64 colours (a plate under 70 cubes) are dropped on both sides alike: the step
  matches the oracle, which drops them the same way.
- jg_device_views hands out the device state arrays; reading them gives jg_query_state's values
  and writing them is what the next step starts from.
"""
import sys

import numpy as np
import pytest

from paper_2606_28394_amd import workloads as W
from parity_util import BAND_MASK, compare_contacts, compare_state, fmt, gpu_manifolds, oracle_manifolds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _towers(n, levels, seed):
    sb = W.SceneBuilder(W.default_params(), 1)
    for t in range(n):
        he, m, pos, quat, _, _ = W.jenga_tower(levels, W.rng_for(seed, t))
        sb.add_tower(he, m, pos, quat, 0.4)
    return sb.build()


def test_nan_tower_is_frozen(J):
    """Six towers in one pack; a NaN velocity in tower 2 freezes that tower only."""
    sc = _towers(6, 7, 71)
    ptr = sc["tower_ptr"]
    a, b = int(ptr[2]), int(ptr[3])
    worlds = [J.World(sc, pack_bodies=250) for _ in range(2)]
    for w in worlds:
        w.step(3)
    x, q, v, om = worlds[0].state()
    vbad = v.copy()
    vbad[a + 4, 1] = np.nan
    worlds[0].set_state(x, q, vbad, om)
    worlds[1].set_state(x, q, v, om)
    for w in worlds:
        w.step(5)
    _say("nan tower: stepping done")
    with pytest.raises(J.JengaError) as ei:
        worlds[0].state()
    assert ei.value.code == J.JG_ENAN
    gx, gq, gv, gw = worlds[0].state()          # reported once: this call returns JG_OK
    rx, rq, rv, rw = worlds[1].state()
    # the frozen tower kept the state it was given, NaN included (jg_set_state normalises the
    # quaternions in double precision, the device holds them in single)
    qq = q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2] + q[:, 3] * q[:, 3]
    qn = (q * (1.0 / np.sqrt(qq))[:, None]).astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(gx[a:b], x[a:b])
    np.testing.assert_array_equal(gq[a:b], qn[a:b])
    np.testing.assert_array_equal(gv[a:b], vbad[a:b])
    np.testing.assert_array_equal(gw[a:b], om[a:b])
    assert np.all(worlds[0].active()[a:b] == 1)
    # every other tower steps exactly as without it
    keep = np.r_[0:a, b:len(gx)]
    for g, r in ((gx, rx), (gq, rq), (gv, rv), (gw, rw)):
        np.testing.assert_array_equal(g[keep], r[keep])
    s = worlds[0].stats()
    assert s.error_word & J.JG_ERR_NAN
    assert len(worlds[0].contacts(2)) == 0 and len(worlds[0].contacts(3)) == len(worlds[1].contacts(3))
    # a finite state from the host unfreezes it
    worlds[0].set_state(rx, rq, rv, rw)
    worlds[1].set_state(rx, rq, rv, rw)
    for w in worlds:
        w.step(2)
    for g, r in zip(worlds[0].state(), worlds[1].state()):
        np.testing.assert_array_equal(g, r)
    for w in worlds:
        w.close()


def test_manifold_capacity_overflow_keeps_canonical_prefix(J, oracle):
    """A 12-level tower (102 colliding pairs) with room for 36 manifolds: the kept pairs are the
    first 36 of the oracle's canonical list."""
    sc = _towers(1, 12, 72)
    nb = int(sc["tower_ptr"][-1])
    gw = J.World(sc, manifolds_per_body=1.0)
    ow = oracle.OracleWorld(sc)
    gw.step(1)
    ow.step(1)
    with pytest.raises(J.JengaError) as ei:
        gw.stats()
    assert ei.value.code == J.JG_ECAPACITY
    s = gw.stats()
    assert s.error_word & J.JG_ERR_MANIFOLDS and not s.error_word & J.JG_ERR_NAN
    om = oracle_manifolds(ow, 0)
    canon = sorted(om, key=lambda k: (k[0], k[1] if k[1] >= 0 else 1 << 30))
    cap = max(16, int(np.ceil(1.0 * nb)))
    assert len(canon) > cap
    assert not any(om[k]["band"] & BAND_MASK for k in canon[:cap + 4])
    gm = gpu_manifolds(gw.contacts(0), 0)
    _say("capacity overflow:", len(canon), "pairs,", len(gm), "kept, capacity", cap)
    assert sorted(gm, key=lambda k: (k[0], k[1] if k[1] >= 0 else 1 << 30)) == canon[:cap]
    assert s.manifolds == cap            # the kept pairs
    gw.close()


def test_colour_cap_drops_like_the_oracle(J, oracle):
    """A plate on the ground under 70 cubes: 71 manifolds share the plate, so greedy colouring
    runs out of its 64 colours; both sides drop the rest and the step matches."""
    he = [[0.5, 0.5, 0.01]] + [[0.02, 0.02, 0.02]] * 70
    mass = [10.0] + [0.1] * 70
    pos = [[0.0, 0.0, 0.01 - 1e-4]]
    pos += [[-0.45 + 0.1 * (k % 10), -0.3 + 0.1 * (k // 10), 0.02 - 2e-4 + 0.02] for k in range(70)]
    n = len(pos)
    sb = W.SceneBuilder(W.default_params(), 1)
    sb.add_tower(np.array(he), np.array(mass), np.array(pos), np.tile([1.0, 0, 0, 0], (n, 1)), 0.5,
                 np.zeros((n, 3)), np.zeros((n, 3)))
    sc = sb.build()
    gw = J.World(sc)
    ow = oracle.OracleWorld(sc)
    gw.step(1)
    ow.step(1)
    with pytest.raises(J.JengaError) as ei:
        gw.sync()
    assert ei.value.code == J.JG_ECAPACITY
    s = gw.stats()
    assert s.error_word & J.JG_ERR_COLOURS and s.colours == 64
    assert ow.tower_stats(0).error & 1
    om = oracle_manifolds(ow, 0)
    gm = gpu_manifolds(gw.contacts(0), 0)
    assert len(om) == 64 and set(gm) == set(om)
    rep = compare_contacts(om, gm, masses=np.array(mass))
    assert rep["ok"], fmt(rep)
    st = compare_state(ow, *gw.state())
    assert st["ok"], st
    gw.close()


def test_device_views_are_the_state(J):
    import torch
    sc = _towers(3, 5, 73)
    gw = J.World(sc)
    ref = J.World(sc)
    gw.step(4)
    ref.step(4)
    views, slots = gw.device_views()
    torch.cuda.synchronize()
    x, q, v, w = gw.state()
    for name, host in (("x", x), ("q", q), ("v", v), ("w", w)):
        dv = views[name].cpu().numpy()[:, slots].T
        np.testing.assert_array_equal(dv, host.astype(np.float32))
    # a write through the view is what the next step starts from (same as jg_set_state)
    body = 7
    views["v"][0, int(slots[body])] += 0.05
    torch.cuda.synchronize()
    v2 = v.copy()
    v2[body, 0] = np.float32(np.float32(v[body, 0]) + np.float32(0.05))
    ref.set_state(linvel=v2)       # the other arrays keep their device values
    ref.commit()
    # the view world keeps its warm-start store; a state upload clears the reference's: with the
    # zero start (warm_start 0) that store is unused, so both steps match
    gw.step(3)
    ref.step(3)
    for g, r in zip(gw.state(), ref.state()):
        np.testing.assert_array_equal(g, r)
    gw.close()
    ref.close()
