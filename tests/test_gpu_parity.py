"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU."""
import math
import sys

import numpy as np
import pytest

from paper_2606_28394_amd import workloads as W
from parity_util import LAM_TOL_FALLING, compare_contacts, compare_state, fmt, gpu_manifolds, oracle_manifolds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# residuals after the sweeps of one step: the RMS and the max over rows of the natural-map
# residual (Sec. "PGS Iterations"); measured on the cases below they agree with the oracle's to
# 9e-6 relative at worst, and 1e-4 leaves a tenfold margin
RES_TOL = 1e-4


def _one_step_compare(J, oracle, scene, states, warm_start=0, n_check_towers=None, label="", pack_bodies=0,
                      lam_tol=1e-4):
    """For each oracle state: put it on the GPU, step once on both sides, compare (impulses to
    lam_tol, relative with the m g dt / 4 floor)."""
    ow = oracle.OracleWorld(scene, warm_start=warm_start)
    gw = J.World(scene, warm_start=warm_start, pack_bodies=pack_bodies)
    ptr = scene["tower_ptr"]
    towers = range(scene["n_towers"]) if n_check_towers is None else range(min(n_check_towers, scene["n_towers"]))
    reports = []
    for (x, q, v, w, act) in states:
        ow.set_state(x, q, v, w)
        ow.active[:] = act
        gw.set_state(x, q, v, w)
        for i in range(len(act)):
            if act[i] == 0:
                J.jg_set_active(gw.h, i, 0)
        ow.step(1)
        gw.step(1)
        assert gw.stats().error_word == 0, f"{label}: device error word {gw.stats().error_word}"
        gx, gq, gv, gww = gw.state()
        st = compare_state(ow, gx, gq, gv, gww)
        worst = 0.0
        for t in towers:
            rep = compare_contacts(oracle_manifolds(ow, t), gpu_manifolds(gw.contacts(t), int(ptr[t])),
                                   lam_tol=lam_tol)
            reports.append((t, rep))
            assert rep["ok"], f"{label} tower {t}: {fmt(rep)}"
            # the residual of the solve (natural map of every PGS row, RMS and max over rows)
            ot, gt = ow.tower_stats(t), gw.stats(t)
            for o, g in ((ot.res_rms, gt.residual_rms), (ot.res_max, gt.residual_max)):
                worst = max(worst, abs(g - o) / (o + 1e-6))
                assert abs(g - o) <= RES_TOL * o + 1e-7, f"{label} tower {t}: residual oracle {o:.6e} gpu {g:.6e}"
        _say(label, "state", st, "residual rel err", f"{worst:.2e}")
        assert st["ok"], f"{label}: state {st}"
    gw.close()
    return reports


def _trajectory_states(oracle, scene, steps, warm_start=0):
    ow = oracle.OracleWorld(scene, warm_start=warm_start)
    out = []
    done = 0
    for s in steps:
        if s > done:
            ow.step(s - done)
            done = s
        out.append((ow.x.copy(), ow.q.copy(), ow.v.copy(), ow.w.copy(), ow.active.copy()))
    return out


def test_free_flight_matches_closed_form(J, oracle):
    v0 = np.array([0.3, -0.2, 0.5])
    w0 = np.array([3.0, -7.0, 11.0])
    q0 = W.quat_axis_angle([1, 2, 3], 0.7)
    x0 = np.array([0.1, 0.2, 5.0])
    sc = W.single_box(x0, q0, v0, w0)
    gw = J.World(sc)
    ow = oracle.OracleWorld(sc)
    gw.step(1)
    gw.step(9)
    gw.step(50)
    ow.step(60)
    gx, gq, gv, gww = gw.state()
    n = 60
    dt = 1 / 240
    x_exp = x0 + n * dt * v0 + np.array([0, 0, -9.81]) * dt * dt * n * (n + 1) / 2
    assert np.abs(gx[0] - x_exp).max() < 1e-5 * 5.0
    st = compare_state(ow, gx, gq, gv, gww)
    _say("free flight", st)
    assert st["x"] < 1e-5 and st["q"] < 1e-4 and st["v"] < 1e-4 and st["w"] < 1e-3
    gw.close()


def test_cfg1_tower_one_step_parity_along_trajectory(J, oracle):
    sc = W.cfg1(0)
    states = _trajectory_states(oracle, sc, [0, 1, 30, 90, 180, 239])
    reps = _one_step_compare(J, oracle, sc, states, label="cfg1")
    assert all(r["pairs"] > 50 for _, r in reps)


def test_tilted_batch_one_step_parity(J, oracle):
    """Towers of up to 40 levels in mid-fall: the impulses are held to 2e-4, twice the bound on the
    single-precision oracle's spread against its FP64 self on this batch (pinned on the CPU by
    test_falling_impulse_spread_is_fp32_arithmetic)."""
    sc = W.tilted_towers(31, 24, levels_range=(8, 40))
    states = _trajectory_states(oracle, sc, [0, 60, 150])
    _one_step_compare(J, oracle, sc, states, label="tilted", lam_tol=LAM_TOL_FALLING)


def test_substeps_one_step_parity(J, oracle):
    """n_sub = 3 substeps of dt / 3 per step and 14 iterations (the paper's own settings): every
    substep runs the whole pipeline on both sides."""
    sc = dict(W.tilted_towers(35, 12, levels_range=(8, 24)))
    sc["params"] = dict(sc["params"], n_sub=3, iters=14)
    states = _trajectory_states(oracle, sc, [0, 40, 100])
    reps = _one_step_compare(J, oracle, sc, states, label="n_sub=3")
    assert all(r["pairs"] > 20 for _, r in reps)


def test_small_towers_many_per_pack(J, oracle):
    """Short towers (8-12 levels): several towers share one on-chip pack (a small batch gets one
    tower per pack by default, so the pack size is set)."""
    sc = W.tilted_towers(32, 40, levels_range=(8, 12))
    states = _trajectory_states(oracle, sc, [0, 80])
    _one_step_compare(J, oracle, sc, states, label="small", pack_bodies=120)


def test_warm_start_parity(J, oracle):
    he, m, pos, quat, lev, slot = W.jenga_tower(18, W.rng_for(33, 0))
    sb = W.SceneBuilder(W.default_params(), 10)
    sb.add_tower(he, m, pos, quat, 0.4)
    sc = sb.build()
    ow = oracle.OracleWorld(sc, warm_start=1)
    gw = J.World(sc, warm_start=1)
    for k in range(3):
        ow.step(1)
        gw.step(1)
        rep = compare_contacts(oracle_manifolds(ow, 0), gpu_manifolds(gw.contacts(0), 0))
        st = compare_state(ow, *gw.state())
        _say("warm step", k, st, fmt(rep))
        assert rep["ok"] and st["ok"]
    gw.close()


def test_pushes_and_withdrawal(J, oracle):
    """A lone pushed block slides out and is removed on the same step on both sides."""
    he = W.BLOCK_HALF
    m = W.BLOCK_MASS
    sb = W.SceneBuilder(W.default_params(), 200)
    sb.add_tower([he], [m], [[0, 0, he[2] - 1e-4]], [[1, 0, 0, 0]], 0.4)
    sb.add_push(0, [1.2 * 3 * 0.4 * m * 9.81, 0, 0], 5, 150, 0.02)
    sc = sb.build()
    ow = oracle.OracleWorld(sc)
    gw = J.World(sc)
    o_gone = g_gone = None
    for s in range(200):
        ow.step(1)
        gw.step(1)
        if o_gone is None and ow.active[0] == 0:
            o_gone = s
        if g_gone is None and gw.active()[0] == 0:
            g_gone = s
        if s in (5, 6, 40):
            st = compare_state(ow, *gw.state())
            assert st["ok"], st
    _say("withdrawn at", o_gone, g_gone)
    assert o_gone is not None and o_gone == g_gone
    gw.close()


@pytest.mark.parametrize("mu", W.MU_LEVELS)
@pytest.mark.parametrize("k", [3, 4])
def test_ziglar_lone_block_on_gpu(J, mu, k):
    he = W.BLOCK_HALF
    m = W.BLOCK_MASS
    axis = np.array([1.0, 0, 0]) if k == 3 else np.array([0, 1.0, 0])
    drift = {}
    for s in (0.98, 1.02):
        sb = W.SceneBuilder(W.default_params(), 240)
        sb.add_tower([he], [m], [[0, 0, he[2] - 1e-4]], [[1, 0, 0, 0]], mu)
        sb.add_push(0, s * k * mu * m * 9.81 * axis, 0, 240)
        sb.add_push(0, [0, 0, -(k - 1) * m * 9.81], 0, 240)
        gw = J.World(sb.build())
        gw.step(240)
        drift[s] = float(gw.state()[0][0] @ axis)
        gw.close()
    expect = 0.02 * k * mu * 9.81 * (1 / 240) ** 2 * 240 * 241 / 2
    _say("ziglar", mu, k, drift)
    assert abs(drift[0.98]) < 5e-4 and abs(drift[0.98]) < 0.01 * abs(drift[1.02])
    assert abs(drift[1.02] - expect) / expect < 0.02


def test_determinism(J):
    sc = W.tilted_towers(34, 16, levels_range=(8, 40))
    outs = []
    for rep in range(2):
        gw = J.World(sc)
        gw.step(40)
        outs.append(gw.state())
        gw.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_edge_cases(J, oracle):
    # a world with no towers
    p = J.jg_default_params()
    h = J.jg_create_world(p, 4, 16)
    J.jg_commit(h)
    J.jg_step_batch(h, 3)
    assert J.jg_query_stats(h).steps == 3
    # one static box with a dynamic box resting on it; one inactive body
    he = W.BLOCK_HALF
    m = W.BLOCK_MASS
    J.jg_add_boxes(h, 0, [he, he, he], [0.0, m, m], [[0, 0, 0.2], [0, 0, 0.2 + 0.015 - 1e-4], [0.5, 0, 1.0]],
                   [[1, 0, 0, 0]] * 3)
    J.jg_set_active(h, 2, 0)
    # host-side changes must be committed before a launch: jg_step_batch only launches
    with pytest.raises(J.JengaError) as ei:
        J.jg_step_batch(h, 60)
    assert ei.value.code == J.JG_ESTATE
    J.jg_commit(h)
    J.jg_step_batch(h, 60)
    x, q, v, w = J.jg_query_state(h, 0, 3)
    assert np.allclose(x[0], [0, 0, 0.2])              # static never moves
    assert abs(x[1, 2] - (0.2 + 0.015 - 1e-4)) < 5e-4  # resting on it
    assert np.allclose(x[2], [0.5, 0, 1.0])            # inactive never moves
    c = J.jg_query_contacts(h, 0)
    assert len(c) == 4 and set(c["body_a"]) == {0} and set(c["body_b"]) == {1}
    # bad arguments are rejected, not crashed on
    with pytest.raises(J.JengaError):
        J.jg_set_active(h, 99, 0)
    with pytest.raises(J.JengaError):
        J.jg_add_boxes(h, 3, [he], [m], [[0, 0, 0]], [[1, 0, 0, 0]])     # towers must be dense
    with pytest.raises(J.JengaError):
        J.jg_add_boxes(h, 1, [[-1, 1, 1]], [m], [[0, 0, 0]], [[1, 0, 0, 0]])
    J.jg_destroy_world(h)
    # a 300-body tower does not fit on chip: it is stepped with its state in device memory
    p = J.jg_default_params()
    p.pack_bodies = 600
    h = J.jg_create_world(p, 2, 300)
    he6, m6, pos6, q6, _, _ = W.jenga_tower(100, None)
    J.jg_add_boxes(h, 0, he6, m6, pos6, q6)
    J.jg_commit(h)
    J.jg_step_batch(h, 2)
    s = J.jg_query_stats(h)
    assert s.error_word == 0 and s.steps == 2 and s.points > 0
    # more bodies than the world was created for are refused with JG_ECAPACITY
    with pytest.raises(J.JengaError) as ei:
        J.jg_add_boxes(h, 1, [he], [m], [[1, 0, 0.2]], [[1, 0, 0, 0]])
    assert ei.value.code == J.JG_ECAPACITY
    J.jg_destroy_world(h)


def test_full_throughput_batch_sampled(J, oracle):
    """The 16384-tower throughput batch in the benchmark's launch configuration: one step on
    the GPU, sampled towers recomputed one by one by the oracle."""
    sc = W.cfg3(0)
    gw = J.World(sc)
    gw.step(1)
    gx, gq, gv, gww = gw.state()
    rng = np.random.default_rng(5)
    sample = sorted(rng.choice(sc["n_towers"], size=12, replace=False).tolist())
    sub = W.subset(sc, sample)
    ow = oracle.OracleWorld(sub)
    ow.step(1)
    ptr = sc["tower_ptr"]
    sptr = sub["tower_ptr"]
    for k, t in enumerate(sample):
        a, b = int(ptr[t]), int(ptr[t + 1])
        rep = compare_contacts(oracle_manifolds(ow, k), gpu_manifolds(gw.contacts(t), a))
        assert rep["ok"], f"tower {t}: {fmt(rep)}"
        sa, sb_ = int(sptr[k]), int(sptr[k + 1])
        ox, oq, ov, oww = ow.x[sa:sb_], ow.q[sa:sb_], ow.v[sa:sb_], ow.w[sa:sb_]
        ex = (np.linalg.norm(ox - gx[a:b], axis=1) / np.maximum(np.linalg.norm(ox, axis=1), 0.075)).max()
        ev = (np.linalg.norm(ov - gv[a:b], axis=1) / np.maximum(np.linalg.norm(ov, axis=1), 9.81 / 240)).max()
        assert ex <= 1e-5 and ev <= 1e-4, (t, ex, ev)
    s = gw.stats()
    _say("full batch stats", s.steps, s.manifolds, s.points, s.colours, s.error_word)
    assert s.error_word == 0
    gw.close()
