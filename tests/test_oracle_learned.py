"""Pins of the oracle's learned warm start inside a step: contact features (closed forms for a
box resting on the ground), the initial-impulse mapping, and the reductions to the plain solve
(a network that predicts zero, and a fallback threshold of zero)."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2606_28394_amd import workloads as W

OVERLAP = 1e-4


def _resting_box(params=None, mu=0.4):
    hz = W.BLOCK_HALF[2]
    return W.single_box([0.0, 0.0, hz - OVERLAP], mu=mu, params=params)


def _zero_net():
    flat = np.zeros(M.SIZE)
    M.unpack(flat)["std"][:] = 1.0
    return flat


def test_features_of_resting_box(oracle):
    sc = _resting_box()
    ow = oracle.OracleWorld(sc)
    ow.step(1, record=True)
    rec = ow.features[0]
    assert rec.shape == (4, oracle.FEAT_RECORD)
    hx, hy, hz = W.BLOCK_HALF
    za = hz - OVERLAP
    gdt = W.G * sc["params"]["dt"]
    m = W.BLOCK_MASS
    I = oracle.box_inertia(m, W.BLOCK_HALF)
    # frame: n = -z, t1 = x, t2 = n x t1 = -y; points are the bottom corners 0..3 halfway to the plane
    for i, slot in enumerate(range(4)):
        sx = 1.0 if slot & 1 else -1.0
        sy = 1.0 if slot & 2 else -1.0
        f = rec[i, :24]
        np.testing.assert_allclose(f[0:3], [za, 0.0, 0.0], atol=1e-15)           # x_B - x_A
        np.testing.assert_array_equal(f[3:7], [1.0, 0.0, 0.0, 0.0])              # q_A^-1 q_B
        np.testing.assert_array_equal(f[7:10], [0.0, 0.0, -1.0])                 # normal
        assert f[10] == pytest.approx(OVERLAP, rel=1e-9)                          # depth
        assert f[11] == 0.4                                                       # mu
        np.testing.assert_array_equal(f[12:15], 0.0)                              # no previous step
        np.testing.assert_allclose(f[15:18], [za + OVERLAP / 2, sx * hx, -sy * hy], rtol=1e-12)  # r_A
        np.testing.assert_allclose(f[18:21], [OVERLAP / 2, sx * hx, -sy * hy], rtol=1e-12)       # r_B
        np.testing.assert_allclose(f[21:24], [-gdt, 0.0, 0.0], rtol=1e-12, atol=1e-18)          # v_rel
        # Eq. (keff) along -z for a lever (a, b, c): 1/m + b^2 / I_x + a^2 / I_y
        assert rec[i, 24] == pytest.approx(1.0 / m + hy ** 2 / I[0] + hx ** 2 / I[1], rel=1e-12)


def test_feature_records_carry_solved_impulses(oracle):
    sc = _resting_box(W.default_params(iters=200))
    ow = oracle.OracleWorld(sc)
    ow.step(1, record=True)
    rec = ow.features[0]
    man = ow.manifolds(0)[0]
    np.testing.assert_array_equal(rec[:, 24:27], man["k"])
    np.testing.assert_array_equal(rec[:, 27:30], man["lam"])
    # converged: the normal impulses cancel the step's fall, m g dt in total (Eq. (lambda_n) scales
    # each increment by 1 + e, so its fixed point is a zero normal velocity)
    total = W.BLOCK_MASS * W.G * sc["params"]["dt"]
    assert rec[:, 27].sum() == pytest.approx(total, rel=1e-9)


def test_previous_impulse_feature(oracle):
    """The previous step's impulses enter in the outputs' units: lambda_d k_d / (|g| dt)."""
    sc = _resting_box()
    ow = oracle.OracleWorld(sc)
    ow.step(1, record=True)
    lam1 = ow.features[0][:, 27:30].copy()
    ow.step(1, record=True)
    k2 = ow.features[0][:, 24:27]
    np.testing.assert_allclose(ow.features[0][:, 12:15], lam1 * k2 / (W.G * sc["params"]["dt"]), rtol=1e-14,
                               atol=1e-300)
    # a resting box carries its weight: the dimensionless normal impulses sum to m k_n over its points
    assert ow.features[0][:, 12].sum() == pytest.approx((W.BLOCK_MASS * k2[:, 0]).mean(), rel=1e-2)


def _tower_scene(levels=6, seed=3):
    """Two upright towers (mu 0.4 and 0.25) with small random velocities, so every solve has work."""
    sb = W.SceneBuilder(W.default_params(), 1)
    for t, mu in enumerate((0.4, 0.25)):
        rng = W.rng_for(44, 2 * seed + t)
        he, m, pos, quat, _, _ = W.jenga_tower(levels, rng)
        sb.add_tower(he, m, pos, quat, mu, rng.normal(0, 0.01, (len(m), 3)), rng.normal(0, 0.3, (len(m), 3)))
    return sb.build()


def _run(oracle, sc, steps, **kw):
    ow = oracle.OracleWorld(sc, **kw)
    ow.step(steps, record=True)
    return ow


def test_zero_network_is_previous_step_start(oracle):
    """A network that predicts no change starts from the previous step's impulses: the
    previous-step warm start (up to the unit conversion's rounding)."""
    sc = _tower_scene()
    iters = sc["params"]["iters"]
    prev = _run(oracle, sc, 3, warm_start=1)
    learned = _run(oracle, sc, 3, warm_start=2, mlp=_zero_net(), mlp_iters=iters)
    for a, b, floor in ((learned.x, prev.x, 0.075), (learned.q, prev.q, 1.0), (learned.v, prev.v, W.G / 240)):
        assert (np.abs(a - b) / np.maximum(np.abs(b), floor)).max() < 1e-12
    for t in range(sc["n_towers"]):
        assert learned.tower_stats(t).fallbacks == 0
        assert prev.tower_stats(t).res_rms > 0.0
        np.testing.assert_allclose(learned.features[t][:, 24:], prev.features[t][:, 24:], rtol=1e-10, atol=1e-15)


def test_zero_threshold_always_falls_back(oracle):
    """With a fallback threshold of zero every learned solve is redone plainly: the result is the
    plain solve's, whatever the network predicted."""
    sc = _tower_scene(seed=4)
    plain = _run(oracle, sc, 2)
    net = M.bf16(W.mlp_init(1))
    learned = _run(oracle, sc, 2, warm_start=2, mlp=net, mlp_iters=3, fallback_tau=0.0)
    np.testing.assert_array_equal(learned.x, plain.x)
    np.testing.assert_array_equal(learned.w, plain.w)
    for t in range(sc["n_towers"]):
        st, sp = learned.tower_stats(t), plain.tower_stats(t)
        assert st.fallbacks == 2
        assert st.contact_iters == sp.contact_iters + 3 * sp.points


def test_no_sweeps_keeps_predicted_impulses(oracle):
    """With zero sweeps after the learned start the impulses are the network's mapped outputs:
    lambda_n = max(0, y_n) |g| dt / k_n, tangents clipped to the friction box."""
    sc = _tower_scene(seed=5)
    net = M.bf16(W.mlp_init(2))
    M.unpack(net)["b3"][:] = [1.5, 0.7, -0.2]
    ow = _run(oracle, sc, 1, warm_start=2, mlp=net, mlp_iters=0)
    dt = sc["params"]["dt"]
    for t in range(sc["n_towers"]):
        rec = ow.features[t]
        y, _ = M.forward(net, rec[:, :24], rounding=True)
        lam = M.warm_start(y, rec[:, 24:27], rec[:, 12:15], sc["mu"][t], W.G, dt)
        np.testing.assert_allclose(rec[:, 27:30], lam, rtol=1e-12, atol=1e-18)
        assert (rec[:, 27] > 0).any()
