"""Learned warm start inside the step kernel, and its per-point feature records, against the
oracle (through the C ABI)."""
import sys

import numpy as np
import pytest

from oracle import mlp as M
from paper_2606_28394_amd import workloads as W
from parity_util import (compare_contacts, compare_records, compare_state, fmt, gpu_manifolds, gpu_records,
                         oracle_manifolds, oracle_records)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scene(n_towers=6, seed=0, levels=(6, 14)):
    """Upright towers with small random velocities (so every solve has work), mixed friction."""
    sb = W.SceneBuilder(W.default_params(), 1)
    rng = W.rng_for(45, seed)
    for t in range(n_towers):
        L = int(rng.integers(levels[0], levels[1] + 1))
        he, m, pos, quat, _, _ = W.jenga_tower(L, rng)
        sb.add_tower(he, m, pos, quat, W.MU_LEVELS[t % 3], rng.normal(0, 0.01, (len(m), 3)),
                     rng.normal(0, 0.3, (len(m), 3)))
    return sb.build()


def _net(seed, const=None):
    flat = W.mlp_init(seed)
    P = M.unpack(flat)
    if const is not None:        # a network whose output is the constant b3
        P["W3"][:] = 0.0
        P["b3"][:] = const
    flat[:M.N_TRAINABLE] = M.bf16(flat[:M.N_TRAINABLE])
    return flat


def _pair(J, oracle, sc, gpu_kw, or_kw, steps=1):
    ow = oracle.OracleWorld(sc, **or_kw)
    gw = J.World(sc, record_features=True, **gpu_kw)
    for _ in range(steps):
        ow.step(1, record=True)
        gw.step(1)
    return ow, gw


def _check_records(sc, ow, gw, lam_tol=1e-4, label=""):
    ptr = sc["tower_ptr"]
    for t in range(sc["n_towers"]):
        rep = compare_records(oracle_records(ow, t), gpu_records(gw.contacts(t), gw.features(t), int(ptr[t])),
                              lam_tol=lam_tol)
        assert rep["ok"], f"{label} tower {t}: {rep}"
    _say(label, "records ok; last", {k: round(v, 3) if isinstance(v, float) else v for k, v in rep.items()
                                     if k != "missing"})


def _check_step(sc, ow, gw, label=""):
    ptr = sc["tower_ptr"]
    for t in range(sc["n_towers"]):
        rep = compare_contacts(oracle_manifolds(ow, t), gpu_manifolds(gw.contacts(t), int(ptr[t])))
        assert rep["ok"], f"{label} tower {t}: {fmt(rep)}"
    st = compare_state(ow, *gw.state())
    _say(label, "state", st)
    assert st["ok"], f"{label}: {st}"


def _close(sa, sb, label, tol=1e-6):
    for name, a, b, floor in zip("xqvw", sa, sb, (0.075, 1.0, W.G / 240, 1.0)):
        d = float((np.abs(a - b) / np.maximum(np.abs(a), floor)).max())
        _say(label, name, "max rel diff", d)
        assert d <= tol, (label, name, d)


def test_feature_records_plain(J, oracle):
    """Records of two consecutive plain steps (the second carries previous impulses)."""
    sc = _scene(seed=1)
    ow, gw = _pair(J, oracle, sc, dict(warm_start=0), dict(warm_start=0), steps=2)
    assert gw.stats().error_word == 0
    _check_records(sc, ow, gw, label="plain")
    assert np.abs(gw.features(-1)[:, 12:15]).max() > 0.0
    gw.close()


@pytest.mark.parametrize("warm", [0, 1])
def test_feature_records_multi_step_launch(J, oracle, warm):
    """Records and state after one launch of several steps (the previous impulses carried on
    chip between steps); without a warm start they only feed the features."""
    sc = _scene(seed=12)
    ow = oracle.OracleWorld(sc, warm_start=warm)
    gw = J.World(sc, record_features=True, warm_start=warm)
    ow.step(4, record=True)
    gw.step(4)
    _check_records(sc, ow, gw, label=f"launch4 warm{warm}")
    _check_step(sc, ow, gw, label=f"launch4 warm{warm}")
    gw.close()


def test_feature_records_warm_start(J, oracle):
    sc = _scene(seed=2)
    ow, gw = _pair(J, oracle, sc, dict(warm_start=1), dict(warm_start=1), steps=3)
    _check_records(sc, ow, gw, label="warm")
    _check_step(sc, ow, gw, label="warm")
    gw.close()


def test_all_tower_records_match_per_tower_queries(J):
    sc = _scene(n_towers=9, seed=3)
    gw = J.World(sc, record_features=True)
    gw.step(2)
    per = np.concatenate([gw.features(t) for t in range(sc["n_towers"])])
    allr = gw.features(-1)
    assert allr.shape == per.shape
    key = lambda a: a[np.lexsort(a.T[::-1])]
    np.testing.assert_array_equal(key(allr), key(per))
    gw.close()


@pytest.mark.parametrize("pack", [0, -1], ids=["lds", "device"])
@pytest.mark.parametrize("steps", [1, 3])
def test_constant_network_parity(J, oracle, steps, pack):
    """A network with constant outputs makes the initial impulses exact functions of k and mu and
    of the previous step's impulses (added back to the predicted change): the learned start,
    mlp_iters sweeps and the records then meet the plain tolerances, for on-chip packs and for
    towers kept in device memory (whose network chunks are split over four waves)."""
    sc = _scene(seed=4)
    net = _net(5, const=[0.3, 0.05, -0.02])
    kw = dict(warm_start=2, mlp=net, mlp_iters=4)
    ow, gw = _pair(J, oracle, sc, dict(kw, fallback_tau=1e30, pack_bodies=pack), dict(kw, fallback_tau=float("inf")),
                   steps=steps)
    assert gw.stats().fallbacks == 0
    _check_records(sc, ow, gw, label=f"const{steps}")
    _check_step(sc, ow, gw, label=f"const{steps}")
    st = gw.stats()
    assert st.contact_iters == 4 * st.points
    for t in range(sc["n_towers"]):
        ro, rg = ow.tower_stats(t).res_rms, gw.stats(t).residual_rms
        _say(f"const{steps} tower {t} residual oracle {ro:.4e} gpu {rg:.4e}")
        assert abs(rg - ro) <= 1e-3 * ro + 1e-7, (t, ro, rg)
    gw.close()


def test_network_initial_impulses(J, oracle):
    """With no sweeps after the learned start the solved impulses are the mapped network outputs;
    the matrix-core network (bf16 operands) is held to 1e-2 of the impulse scale."""
    sc = _scene(seed=6)
    net = _net(7)
    M.unpack(net)["b3"][:] = M.bf16(np.array([0.6, 0.1, -0.1]))
    kw = dict(warm_start=2, mlp=net, mlp_iters=0)
    ow, gw = _pair(J, oracle, sc, dict(kw, fallback_tau=1e30), dict(kw, fallback_tau=float("inf")))
    recs = gw.features(-1)
    assert (recs[:, 27] > 0).mean() > 0.2
    _check_records(sc, ow, gw, lam_tol=1e-2, label="net0")
    gw.close()


def test_zero_network_is_previous_step_start_on_gpu(J):
    """No predicted change and iters sweeps: the learned variant reproduces the previous-step warm
    start of the plain kernel (up to the FP32 unit conversion: 1e-5 relative)."""
    sc = _scene(seed=8)
    zero = np.zeros(M.SIZE)
    M.unpack(zero)["std"][:] = 1.0
    prev = J.World(sc, warm_start=1)
    learned = J.World(sc, warm_start=2, mlp=zero, mlp_iters=sc["params"]["iters"])
    prev.step(3)
    learned.step(3)
    _close(prev.state(), learned.state(), "zero net", tol=1e-5)
    assert learned.stats().fallbacks == 0
    for t in range(sc["n_towers"]):
        rp, rl = prev.stats(t).residual_rms, learned.stats(t).residual_rms
        assert rp > 0.0 and abs(rl - rp) <= 1e-3 * rp, (t, rp, rl)
    prev.close()
    learned.close()


def test_zero_threshold_falls_back_to_plain(J, oracle):
    """tau = 0 redoes every tower's solve plainly: the plain kernel's result (3e-6 relative; the
    two kernel instantiations fuse multiply-adds differently outside the solve, so two steps of a
    falling tower drift apart by a few FP32 roundings) and the oracle's within the plain
    tolerances; fallbacks and sweeps are counted."""
    sc = _scene(seed=9)
    net = _net(10)
    plain = J.World(sc)
    learned = J.World(sc, warm_start=2, mlp=net, mlp_iters=3, fallback_tau=0.0)
    plain.step(2)
    learned.step(2)
    _close(plain.state(), learned.state(), "tau0", tol=3e-6)
    st, sp = learned.stats(), plain.stats()
    assert st.fallbacks == 2 * sc["n_towers"]
    assert st.contact_iters == sp.contact_iters + 3 * sp.points
    ow = oracle.OracleWorld(sc, warm_start=2, mlp=net, mlp_iters=3, fallback_tau=0.0)
    ow.step(2)
    _check_step(sc, ow, learned, label="tau0")
    plain.close()
    learned.close()


def test_learned_mode_needs_network(J):
    sc = _scene(n_towers=1, seed=11)
    gw = J.World(sc, warm_start=2)
    with pytest.raises(J.JengaError):
        gw.step(1)
    gw.close()


def test_learned_and_records_in_device_memory_match_lds(J):
    """The learned warm start and the feature records with the layout in device memory
    (pack_bodies = -1) against the LDS path, one step from the same state: the same pairs and
    fallbacks, state and impulses within the parity tolerances, records close."""
    sc = _scene(6, seed=3)
    net = _net(5)
    G_DT = 9.81 / 240.0
    for kw in (dict(warm_start=2, mlp=net, mlp_iters=4, fallback_tau=1e30),
               dict(warm_start=2, mlp=net, mlp_iters=4, fallback_tau=0.0),
               dict(record_features=True)):
        lds = J.World(sc, **kw)
        dev = J.World(sc, pack_bodies=-1, **kw)
        lds.step(1)
        dev.step(1)
        (lx, lq, lv, lw), (dx, dq, dv, dw) = lds.state(), dev.state()
        ex = float((np.linalg.norm(lx - dx, axis=1) / np.maximum(np.linalg.norm(lx, axis=1), 0.075)).max())
        ev = float((np.linalg.norm(lv - dv, axis=1) / np.maximum(np.linalg.norm(lv, axis=1), G_DT)).max())
        ew = float((np.linalg.norm(lw - dw, axis=1) / np.maximum(np.linalg.norm(lw, axis=1), 1.0)).max())
        _say(sorted(kw), "x", ex, "v", ev, "w", ew, "fallbacks", lds.stats().fallbacks, dev.stats().fallbacks)
        assert ex <= 1e-5 and float(np.abs(lq - dq).max()) <= 1e-5 and ev <= 1e-4 and ew <= 1e-4
        assert lds.stats().fallbacks == dev.stats().fallbacks
        ptr = sc["tower_ptr"]
        for t in range(sc["n_towers"]):
            a = int(ptr[t])
            ca, cb = gpu_manifolds(lds.contacts(t), a), gpu_manifolds(dev.contacts(t), a)
            assert set(ca) == set(cb)
            for key in ca:
                assert ca[key]["colour"] == cb[key]["colour"] and ca[key]["slot"] == cb[key]["slot"]
                scale = np.maximum(np.abs(ca[key]["lam"]), float(sc["mass"][a + key[0]]) * G_DT / 4.0)
                assert (np.abs(ca[key]["lam"] - cb[key]["lam"]) / scale).max() <= 2e-4, (t, key)
            if kw.get("record_features"):
                fa, fb = lds.features(t), dev.features(t)
                assert fa.shape == fb.shape
                np.testing.assert_allclose(fa, fb, rtol=1e-4, atol=1e-6)
        lds.close()
        dev.close()


def test_learned_multi_step_device_matches_lds(J):
    """Four steps of the learned start (a random network, no fallback) with the towers kept in
    device memory against on-chip packs: from the second step on the previous impulses enter the
    network's inputs and are added back to its output, on the four waves' own staging rows.  The
    same pairs every step, no fallbacks, each tower's sweeps counted as mlp_iters, and states
    within the one-step parity tolerances times the steps."""
    sc = _scene(6, seed=14)
    net = _net(15)
    kw = dict(warm_start=2, mlp=net, mlp_iters=4, fallback_tau=1e30)
    lds = J.World(sc, **kw)
    dev = J.World(sc, pack_bodies=-1, **kw)
    G_DT = 9.81 / 240.0
    ptr = sc["tower_ptr"]
    for step in range(4):
        lds.step(1)
        dev.step(1)
        (lx, lq, lv, lw), (dx, dq, dv, dw) = lds.state(), dev.state()
        ex = float((np.linalg.norm(lx - dx, axis=1) / np.maximum(np.linalg.norm(lx, axis=1), 0.075)).max())
        ev = float((np.linalg.norm(lv - dv, axis=1) / np.maximum(np.linalg.norm(lv, axis=1), G_DT)).max())
        _say("learned device vs lds, step", step, "x", ex, "v", ev)
        assert ex <= 1e-5 * (step + 1) and float(np.abs(lq - dq).max()) <= 1e-5 * (step + 1)
        assert ev <= 1e-4 * (step + 1)
        for t in range(sc["n_towers"]):
            a = int(ptr[t])
            assert set(gpu_manifolds(lds.contacts(t), a)) == set(gpu_manifolds(dev.contacts(t), a)), (step, t)
    for w in (lds, dev):
        st = w.stats()
        assert st.fallbacks == 0 and st.error_word == 0
        assert st.contact_iters == 4 * st.points
    lds.close()
    dev.close()


def test_island_fallback_with_helper_waves(J):
    """Towers kept in device memory run the learned variant on four waves (the helpers share the
    walk, the manifolds, the network's chunks and the sweeps; the residual and the fallback solve
    stay on the first wave).  With tau = 0 every tower falls back, so three steps must give the
    plain island kernel's result (3e-6 relative, as for on-chip packs), with the fallbacks
    counted."""
    sc = _scene(seed=12)
    net = _net(13)
    plain = J.World(sc, pack_bodies=-1)
    learned = J.World(sc, pack_bodies=-1, warm_start=2, mlp=net, mlp_iters=3, fallback_tau=0.0)
    for w in (plain, learned):
        w.step(1)
        w.step(2)
    _close(plain.state(), learned.state(), "island tau0", tol=3e-6)
    st = learned.stats()
    assert st.error_word == 0 and plain.stats().error_word == 0
    assert st.fallbacks == 3 * sc["n_towers"]
    plain.close()
    learned.close()
