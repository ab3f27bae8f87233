"""Labels of removal episodes and their JSON records.

Each episode of a removal run is one tower. Its labels follow the paper's table of model outputs
(Sec. "Interpreting Predictions") and Tab. results (Sec. "Effect of the Friction Coefficient"):

- num_removed: the blocks withdrawn by the moves started by the collapse step, or by the end of
  the run (jg_episode.removed);
- removed_locs: the tower positions those blocks held, as a levels x 3 map of 0 and 1. It comes
  from the activity flags at the end of the run against those at its start, with each block's
  level and slot from the scene (blocks of a tower built by `workloads.jenga_tower`);
- imbalance_score: minus the support-polygon margin of the centre of mass (Eq. (stability)) at
  the last step before the collapse, in mm (jg_episode.imbalance is in metres; None when the
  first step collapsed);
- torque_risk: the moves across a side block (Tab. ziglar, k = 4) among those moves
  (jg_episode.torque_moves);
- the collapse flag and step, the rounds (moves started), and the step the tower came to rest.

`write_json` stores every episode in one file and one summary per friction level, the layout of
the paper's experiment data. A summary holds:
- the collapsed episodes and the episode count;
- the mean rounds;
- Ziglar's thresholds F_min = 3 mu m g and F_tau = 4 mu m g for the paper's block and for the
  benchmark block;
- the share of torque moves, the mean imbalance and the mean steps from collapse to rest.

Host code only: it reads what the library returns and does no physics.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import workloads as W


def _get(ep, key):
    return ep[key] if isinstance(ep, dict) else getattr(ep, key)


def episode_record(scene: dict, tower: int, ep, active_end) -> dict:
    """The labels of one tower's episode.  ep: a jg_episode (or a dict with its fields);
    active_end: the activity flags of every body of the world at the end of the run."""
    ptr = scene["tower_ptr"]
    a, b = int(ptr[tower]), int(ptr[tower + 1])
    start = np.asarray(scene["active"][a:b]).astype(bool)
    end = np.asarray(active_end[a:b]).astype(bool)
    gone = np.nonzero(start & ~end)[0]
    n_all = len(scene["mass"])
    lev = np.asarray(scene.get("body_level", np.full(n_all, -1)))[a:b]
    slot = np.asarray(scene.get("body_slot", np.full(n_all, -1)))[a:b]
    levels = int(lev.max()) + 1 if (lev >= 0).any() else 0
    locs = np.zeros((levels, 3), np.int8)
    for i in gone:
        if lev[i] >= 0 and 0 <= slot[i] < 3:
            locs[lev[i], slot[i]] = 1
    collapsed = bool(_get(ep, "collapsed"))
    rest = int(_get(ep, "rest_step"))
    imb = float(_get(ep, "imbalance"))
    return {
        "tower": int(tower),
        "mu": float(scene["mu"][tower]),
        "levels": levels,
        "collapsed": collapsed,
        "collapse_step": int(_get(ep, "collapse_step")) if collapsed else None,
        "rest_step": rest if rest >= 0 else None,
        "rounds": int(_get(ep, "rounds")),
        "num_removed": int(_get(ep, "removed")),
        "removed_locs": locs.tolist(),
        "removed_bodies": [int(a + i) for i in gone],
        "imbalance_score_mm": 1e3 * imb if math.isfinite(imb) else None,
        "torque_risk": int(_get(ep, "torque_moves")),
    }


def world_records(world, scene: dict) -> list:
    """Every tower's record from a GPU world after its episode launch (jenga.World)."""
    active = np.asarray(world.active())
    return [episode_record(scene, t, world.episode(t), active) for t in range(scene["n_towers"])]


def _mean(xs):
    xs = [x for x in xs if x is not None]
    return float(np.mean(xs)) if xs else None


def summary(records: list) -> list:
    """One row per friction level of the records (Tab. results)."""
    rows = []
    for mu in sorted({r["mu"] for r in records}):
        rs = [r for r in records if r["mu"] == mu]
        col = [r for r in rs if r["collapsed"]]
        rounds = sum(r["rounds"] for r in rs)
        rows.append({
            "mu": mu,
            "collapsed": len(col),
            "episodes": len(rs),
            "mean_rounds": float(np.mean([r["rounds"] for r in rs])),
            "removed": int(sum(r["num_removed"] for r in rs)),
            "F_min_mN": 3 * mu * W.PAPER_BLOCK_MASS * W.G * 1e3,
            "F_tau_mN": 4 * mu * W.PAPER_BLOCK_MASS * W.G * 1e3,
            "F_min_mN_benchmark_block": 3 * mu * W.BLOCK_MASS * W.G * 1e3,
            "torque_move_pct": 100.0 * sum(r["torque_risk"] for r in rs) / max(1, rounds),
            "mean_imbalance_mm": _mean([r["imbalance_score_mm"] for r in rs]),
            "mean_steps_to_rest": _mean([r["rest_step"] - r["collapse_step"] for r in col
                                         if r["rest_step"] is not None]),
        })
    return rows


def write_json(records: list, directory: str, tag: str = "") -> list:
    """episodes{tag}.json with every record and summary_mu{mu}{tag}.json per friction level;
    returns the paths written."""
    os.makedirs(directory, exist_ok=True)
    paths = [os.path.join(directory, f"episodes{tag}.json")]
    with open(paths[0], "w") as f:
        json.dump(records, f, indent=1)
    for row in summary(records):
        p = os.path.join(directory, f"summary_mu{row['mu']:.2f}{tag}.json")
        with open(p, "w") as f:
            json.dump(row, f, indent=1)
        paths.append(p)
    return paths
