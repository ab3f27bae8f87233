"""Episode labels and their JSON records (the episode layer's host code), from given episode
results: the map of removed positions, the per-friction summary rows against the thresholds
printed in Tab. results, and the JSON round trip."""
import json
import math

import numpy as np

from paper_2606_28394_amd import episodes as E
from paper_2606_28394_amd import workloads as W


def _scene():
    return W.cfg2(0, n_per_mu=2, n_steps=10)   # 6 towers of 12-24 levels, with their level / slot


def _ep(**kw):
    base = dict(collapsed=0, collapse_step=-1, rest_step=-1, rounds=0, removed=0, imbalance=float("nan"),
                torque_moves=0)
    base.update(kw)
    return base


def test_removed_locs_map_positions():
    sc = _scene()
    ptr = sc["tower_ptr"]
    t = 1
    a, b = int(ptr[t]), int(ptr[t + 1])
    active = np.asarray(sc["active"]).copy()
    for lev, slot in ((3, 1), (5, 2)):   # the centre block of layer 3, a side block of layer 5
        active[a + 3 * lev + slot] = 0
    active[int(ptr[2])] = 0              # another tower's block: not this tower's label
    r = E.episode_record(sc, t, _ep(rounds=2, removed=2, torque_moves=1), active)
    locs = np.array(r["removed_locs"])
    assert locs.shape == ((b - a) // 3, 3) and r["levels"] == (b - a) // 3
    assert locs.sum() == 2 and locs[3, 1] == 1 and locs[5, 2] == 1
    assert r["removed_bodies"] == [a + 10, a + 17]
    assert r["num_removed"] == 2 and r["torque_risk"] == 1 and r["rounds"] == 2
    assert r["collapse_step"] is None and r["rest_step"] is None and r["imbalance_score_mm"] is None
    # a block already missing at the start (cfg1's removed block) is not a removal of the episode
    s1 = W.cfg1(0)
    r1 = E.episode_record(s1, 0, _ep(), np.asarray(s1["active"]))
    assert r1["num_removed"] == 0 and np.array(r1["removed_locs"]).sum() == 0 and r1["levels"] == 18
    # subsets keep the positions
    sub = W.subset(sc, [t])
    r2 = E.episode_record(sub, 0, _ep(removed=2), active[a:b])
    assert r2["removed_locs"] == r["removed_locs"]


def test_collapse_fields_and_units():
    sc = _scene()
    r = E.episode_record(sc, 0, _ep(collapsed=1, collapse_step=412, rest_step=530, imbalance=0.0123, rounds=3),
                         np.asarray(sc["active"]))
    assert r["collapsed"] and r["collapse_step"] == 412 and r["rest_step"] == 530
    assert abs(r["imbalance_score_mm"] - 12.3) < 1e-9


def test_summary_rows_match_table_thresholds():
    """Ziglar's thresholds in the summary are the ones Tab. results prints for the paper's block
    (F_min 144.2 / 230.7 / 346.1 mN, F_tau 192.3 / 307.6 / 461.5 mN at mu = 0.25 / 0.40 / 0.60)."""
    sc = W.cfg2(0, n_per_mu=2, n_steps=10)
    act = np.asarray(sc["active"])
    eps = [_ep(collapsed=int(t % 2 == 0), collapse_step=100 + t, rest_step=(200 + t) if t % 4 == 0 else -1,
               rounds=t + 1, torque_moves=t % 2, removed=t % 3, imbalance=0.001 * t) for t in range(6)]
    recs = [E.episode_record(sc, t, eps[t], act) for t in range(6)]
    rows = E.summary(recs)
    assert [r["mu"] for r in rows] == list(W.MU_LEVELS)
    printed = {0.25: (144.2, 192.3), 0.40: (230.7, 307.6), 0.60: (346.1, 461.5)}
    for row in rows:
        fmin, ftau = printed[row["mu"]]
        assert abs(row["F_min_mN"] - fmin) < 0.05 and abs(row["F_tau_mN"] - ftau) < 0.05
        ts = [t for t in range(6) if sc["mu"][t] == row["mu"]]
        assert row["episodes"] == 2 and row["collapsed"] == sum(t % 2 == 0 for t in ts)
        assert row["mean_rounds"] == np.mean([t + 1 for t in ts])
        assert row["removed"] == sum(t % 3 for t in ts)
        assert math.isclose(row["torque_move_pct"], 100.0 * sum(t % 2 for t in ts) / sum(t + 1 for t in ts))
        rest = [100 for t in ts if t % 2 == 0 and t % 4 == 0]   # rest_step - collapse_step
        assert row["mean_steps_to_rest"] == (float(np.mean(rest)) if rest else None)


def test_json_round_trip(tmp_path):
    sc = _scene()
    act = np.asarray(sc["active"]).copy()
    act[int(sc["tower_ptr"][3]) + 4] = 0
    recs = [E.episode_record(sc, t, _ep(removed=int(t == 3), rounds=1), act) for t in range(sc["n_towers"])]
    paths = E.write_json(recs, str(tmp_path), tag="_test")
    assert len(paths) == 1 + len(W.MU_LEVELS)
    with open(paths[0]) as f:
        back = json.load(f)
    assert back == recs
    with open(paths[1]) as f:
        row = json.load(f)
    assert row == E.summary(recs)[0]
