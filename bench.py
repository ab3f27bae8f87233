"""Throughput benchmark of batched tower stepping on one MI355X.

Workload (default): the throughput batch -- 16384 towers of 8-40 levels x 3 boxes
(75 x 25 x 15 mm, 600 kg/m^3), each tilted past its critical angle about a seeded
bottom edge so it collapses fully; mu_s drawn from {0.25, 0.40, 0.60}; dt = 1/240 s,
20 PGS iterations, FP32 on the GPU.  One bench "step" advances every tower by one
time step through the whole path (broadphase, SAT, manifolds, colouring, PGS,
residual, integration, position correction).

The K timed steps run as one persistent launch (jg_step_batch(world, K)) from the
batch's initial state, with every input already resident in HBM; W warm-up steps run
first and the initial state is then restored.  Before that, the pack-size tuner
(paper_2606_28394_amd/autotune.py) times a few pack sizes on the batch and the timed
world uses its choice.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (published)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2606_28394_amd/csrc/jenga_step.hip", "paper_2606_28394_amd/csrc/jenga_device.h",
                  "paper_2606_28394_amd/csrc/jenga_world.hip"]   # the kernels and the launch layout


def log(*a):
    print(*a, file=sys.stderr, flush=True)


DEVICE_ERRORS = []   # device error reports (capacity, non-finite state) met by any leg
RUN = [""]           # the run the next syncing call belongs to, named in its report


def _synced(J, fn, *a):
    """A syncing C-ABI query; device error bits it reports (JG_ECAPACITY / JG_ENAN: the call did
    its work) are noted in the output instead of ending the run."""
    try:
        return fn(*a)
    except J.JengaError as e:
        if e.code in (J.JG_ECAPACITY, J.JG_ENAN) and e.result is not None:
            DEVICE_ERRORS.append(f"{RUN[0]}: {e}" if RUN[0] else str(e))
            log(f"  device error report: {e}")
            return e.result
        raise


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_flops(n_bodies_per_tower, steps, candidates, manifolds, points, iters):
    """FP32 operations the method needs (not what the kernel executes), summed over a launch:
    per tower-step 250 N (frames, integration) + 12 N(N-1)/2 (AABB tests) + 350 per candidate
    (SAT) + 1200 per manifold (projection, clipping) + 210 per point (prep) + 156 per point and
    iteration (three PGS rows) + 90 per point (residual)."""
    pair_tests = sum(12.0 * n * (n - 1) / 2 + 250.0 * n for n in n_bodies_per_tower) * steps
    return pair_tests + 350.0 * candidates + 1200.0 * manifolds + (210.0 + 156.0 * iters + 90.0) * points


def algorithmic_bytes(n_bodies_total, n_points_launch_end):
    """HBM bytes one launch must move: body state in and out (13 floats each way + 5 static
    words read) and the final contacts written (32 B per point)."""
    return n_bodies_total * (13 * 4 * 2 + 5 * 4) + 32.0 * n_points_launch_end


def traffic_from_profile(khash: str, workload: str, steps: int, pack_bodies: int = 0):
    """HBM bytes of one launch of `steps` steps from the committed counter record (FETCH_SIZE +
    WRITE_SIZE of a launch of the same batch).  Nearly all of it is per step (the contact points'
    lever arms and impulses stream through device memory on every sweep), so the record scales
    with the step count; a changed kernel invalidates it."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != khash or not workload.startswith(rec.get("workload", "\0")):
        return None
    if int(rec.get("pack_bodies", 0)) != pack_bodies:   # counters taken with another packing
        return None
    return rec["hbm_bytes_per_launch"] * steps / rec["steps"]


def cpu_baseline(scene, n_towers=1024, n_steps=50, threads=None):
    """The FP64 oracle on the host cores over a bounded sample of the same batch."""
    from oracle import oracle as O
    from paper_2606_28394_amd import workloads as W
    threads = threads or min(16, os.cpu_count() or 1)
    sub = W.subset(scene, range(min(n_towers, scene["n_towers"])))
    ow = O.OracleWorld(sub)
    t0 = time.perf_counter()
    ow.step(n_steps, threads=threads)
    dt = time.perf_counter() - t0
    ci = sum(ow.tower_stats(t).contact_iters for t in range(sub["n_towers"]))
    return dict(value=sub["n_towers"] * n_steps / dt, unit="tower-steps/s", cores=threads, kind="oracle",
                sample=f"first {sub['n_towers']} towers x {n_steps} steps of the same batch, FP64, "
                       f"{threads} threads, {dt:.1f} s",
                contact_iters_per_s=ci / dt)


def cpu_report(threads=None):
    """The FP64 oracle on one host thread and on all of them, over bounded samples of the four
    workloads: the 18-level removal tower (240 steps), the removal batch (450 towers x 200 steps),
    the throughput batch (first 1024 towers x 50 steps) and the 64 x 64 wall (100 steps; one
    island, so one thread does the work either way)."""
    from oracle import oracle as O
    from paper_2606_28394_amd import workloads as W
    threads = threads or min(16, os.cpu_count() or 1)
    samples = [("removal tower, 240 steps", W.cfg1(0), 240),
               ("removal batch, 450 towers x 200 steps", W.cfg2(0, n_steps=200), 200),
               ("throughput batch, first 1024 towers x 50 steps", W.subset(W.cfg3(0, n_steps=50), range(1024)), 50),
               ("masonry wall, 100 steps", W.cfg5(0, n_steps=100), 100)]
    out = []
    for name, sc, n in samples:
        row = dict(sample=name, towers=sc["n_towers"], bodies=int(sc["tower_ptr"][-1]), steps=n)
        for th in (1, threads):
            ow = O.OracleWorld(sc)
            t0 = time.perf_counter()
            ow.step(n, threads=th)
            dt = time.perf_counter() - t0
            ci = sum(ow.tower_stats(t).contact_iters for t in range(sc["n_towers"]))
            row[f"threads_{th}"] = dict(tower_steps_per_s=sc["n_towers"] * n / dt, contact_iters_per_s=ci / dt,
                                        seconds=dt)
            log(f"  oracle {name}, {th} thread(s): {sc['n_towers'] * n / dt:.4g} tower-steps/s ({dt:.1f} s)")
        out.append(row)
    return dict(cores=threads, samples=out)


DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_2606_28394_amd", "data", "warmstart_mlp.npy")


def _run_residuals(J, scene, steps, chunk, run="", **kw):
    """Step a fresh world `steps` steps in launches of `chunk`; median and mean of the per-tower
    residual (RMS over rows) at each launch end, and the counters.  run: names the run in device
    error reports."""
    import numpy as np
    RUN[0] = run
    world = J.World(scene, **kw)
    res = []
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        world.step(n)
        done += n
        res.extend(_synced(J, world.stats, t).residual_rms for t in range(scene["n_towers"]))
    st = _synced(J, world.stats)
    world.close()
    res = np.asarray(res)
    return float(np.median(res)), float(res.mean()), st


def _run_timed(J, torch, scene, steps, keep=False, run="", **kw):
    """One persistent launch of `steps` steps from the initial state; tower-steps/s from HIP events.
    keep: return the open world with the stats, (world, stats), instead of closing it.  run: names
    the run in device error reports."""
    RUN[0] = run
    stream = torch.cuda.current_stream()
    world = J.World(scene, stream=stream.cuda_stream, **kw)
    world.step(0)
    world.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    world.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = _synced(J, world.stats)
    if keep:
        return scene["n_towers"] * steps / (ms * 1e-3), ms, (world, st)
    world.close()
    return scene["n_towers"] * steps / (ms * 1e-3), ms, st


def equal_residual(J, torch, weights, steps=2000, chunk=50, ks=(1, 2, 4, 8, 12), scene=None, workload=None):
    """The learned warm start against plain PGS at 20 iterations at equal residual, on the
    450-tower removal batch (or `scene`).  R20 = median tower residual of plain-20.  For each k:
    - the learned start alone (no fallback, tau = inf): median residual and rate;
    - the learned start with the fallback at tau = R20 (a tower above it is solved again
      plainly): median residual, fallback share, sweeps per point, rate;
    - the previous-step start (no network) at k sweeps: median residual and rate.
    The learned equal-residual point is the smallest k whose learned-alone median is <= R20; the
    fallback run counts only where its sweeps per point stay below plain-20's (else the residual
    is mostly the plain solver's).  Rates include inference, residual passes and fallbacks."""
    import numpy as np
    from paper_2606_28394_amd import workloads as W
    net = np.load(weights)
    if scene is None:
        scene = W.cfg2(0, n_steps=steps)
        workload = (f"removal batch: {scene['n_towers']} towers, 12-24 levels, 1-8 push removals each, "
                    f"{steps} steps")
    iters = int(scene["params"]["iters"])
    tag = workload.split(":")[0].split(",")[0]
    r20, m20, st20 = _run_residuals(J, scene, steps, chunk, run=f"{tag}, plain-20")
    v20, ms20, _ = _run_timed(J, torch, scene, steps, run=f"{tag}, plain-20")
    log(f"plain-20: median residual {r20:.3e} m/s, {v20:.4g} tower-steps/s")
    alone, fallback, prev_rows, ctx = [], [], [], {}
    for k in ks:
        kw = dict(warm_start=2, mlp=net, mlp_iters=k)
        run = f"{tag}, learned start alone, k={k}"
        rk, mk, _ = _run_residuals(J, scene, steps, chunk, fallback_tau=1e30, run=run, **kw)
        vk, msk, _ = _run_timed(J, torch, scene, steps, fallback_tau=1e30, run=run, **kw)
        alone.append(dict(k=k, median_residual=rk, mean_residual=mk, value=vk, kernel_ms=msk))
        run = f"{tag}, learned start with fallback, k={k}"
        rf, mf, _ = _run_residuals(J, scene, steps, chunk, fallback_tau=r20, run=run, **kw)
        vf, msf, stf = _run_timed(J, torch, scene, steps, fallback_tau=r20, run=run, **kw)
        fallback.append(dict(k=k, median_residual=rf, mean_residual=mf, value=vf, kernel_ms=msf,
                             fallback_rate=stf.fallbacks / (scene["n_towers"] * steps),
                             contact_iters_per_point=stf.contact_iters / max(1, stf.points)))
        p = dict(scene["params"])
        p["iters"] = k
        ctx[f"zero_k{k}"] = _run_residuals(J, scene, steps, chunk, params=p, run=f"{tag}, zero start, k={k}")[0]
        run = f"{tag}, previous-step start, k={k}"
        rp, mp, _ = _run_residuals(J, scene, steps, chunk, params=p, warm_start=1, run=run)
        vp, msp, _ = _run_timed(J, torch, scene, steps, params=p, warm_start=1, run=run)
        prev_rows.append(dict(k=k, median_residual=rp, mean_residual=mp, value=vp, kernel_ms=msp))
        log(f"k={k}: learned alone {rk:.3e} ({vk:.4g}/s); with fallback {rf:.3e} "
            f"({100 * fallback[-1]['fallback_rate']:.1f}% fall back, {vf:.4g}/s); previous step {rp:.3e} ({vp:.4g}/s)")

    def first(rows, ok):
        good = [r for r in rows if ok(r)]
        return min(good, key=lambda r: r["k"]) if good else None

    best = first(alone, lambda r: r["median_residual"] <= r20)
    bestf = first(fallback, lambda r: r["median_residual"] <= r20 and r["contact_iters_per_point"] < iters)
    bestp = first(prev_rows, lambda r: r["median_residual"] <= r20)
    return dict(workload=workload,
                plain20=dict(median_residual=r20, mean_residual=m20, value=v20, kernel_ms=ms20),
                learned_alone=alone, learned_with_fallback=fallback, previous_step=prev_rows,
                median_residual_zero_start=ctx,
                equal_residual_k=best["k"] if best else None,
                learned_vs_plain20=(best["value"] / v20) if best else None,
                fallback_equal_residual_k=bestf["k"] if bestf else None,
                fallback_vs_plain20=(bestf["value"] / v20) if bestf else None,
                previous_step_equal_residual_k=bestp["k"] if bestp else None,
                previous_step_vs_plain20=(bestp["value"] / v20) if bestp else None,
                learned_vs_previous_step=(best["value"] / bestp["value"]) if best and bestp else None)


def large_island(J, torch, W, steps):
    """One 4,096-stone wall (a single island, kept in device memory), plain PGS-20: time per step
    from HIP events over one launch of `steps` steps after 5 warm-up steps."""
    scene = W.cfg5(0, n_steps=steps + 5)
    stream = torch.cuda.current_stream()
    world = J.World(scene, stream=stream.cuda_stream)
    world.step(5)
    _synced(J, world.sync)
    s0 = _synced(J, world.stats)
    _synced(J, J.jg_query_phase_cycles, world.h)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    world.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s1 = _synced(J, world.stats)
    phases = _synced(J, J.jg_query_phase_cycles, world.h)
    tot = max(1, sum(phases.values()))
    n = int(scene["tower_ptr"][-1])
    world.close()
    log(f"  {steps} steps: {ms / steps:.2f} ms per step")
    return {"workload": f"one masonry wall, 64 courses x 64 stones ({n} bodies), steps 6-{5 + steps}",
            "steps": steps, "ms_per_step": ms / steps, "body_steps_per_s": n * steps / (ms * 1e-3),
            "manifolds_per_step": (s1.manifolds - s0.manifolds) / steps,
            "points_per_step": (s1.points - s0.points) / steps,
            "phase_cycle_share": {k: round(v / tot, 4) for k, v in phases.items()},
            "error_word": int(s1.error_word)}


def grid_wide_islands(J, torch, W, steps=10):
    """Islands stepped by the whole GPU (one cooperative launch, grid-wide phases): the
    100,000-stone wall (100 courses x 1,000 stones; the default path for islands of 16,384 bodies or
    more) and the 4,096-stone wall put on the same path (mega_bodies 1,024) to set beside its
    one-workgroup figure.  Time per step from HIP events over one launch of `steps` steps after 2."""
    out = {}
    for key, scene in (("site_wall_100k", W.masonry_wall(100, 1000, seed=0, n_steps=steps + 2)),
                       ("wall_4096", W.cfg5(0, n_steps=steps + 2))):
        if key == "wall_4096":
            scene = dict(scene, params=dict(scene["params"], mega_bodies=1024))
        stream = torch.cuda.current_stream()
        world = J.World(scene, stream=stream.cuda_stream)
        world.step(2)
        _synced(J, world.sync)
        s0 = _synced(J, world.stats)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        world.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        s1 = _synced(J, world.stats)
        n = int(scene["tower_ptr"][-1])
        world.close()
        log(f"  {key}: {ms / steps:.2f} ms per step")
        out[key] = {"bodies": n, "steps": steps, "ms_per_step": ms / steps,
                    "body_steps_per_s": n * steps / (ms * 1e-3),
                    "manifolds_per_step": (s1.manifolds - s0.manifolds) / steps,
                    "points_per_step": (s1.points - s0.points) / steps,
                    "contact_iters_per_s": (s1.contact_iters - s0.contact_iters) / (ms * 1e-3),
                    "colours": int(s1.colours), "error_word": int(s1.error_word)}
    out["workload"] = ("one island per world, plain PGS-20, zero start, steps 3-" + str(2 + steps) +
                       "; partitions of 1,024 stones for the colouring")
    return out


def single_tower_latency(J, torch, W):
    """The 18-level tower with one middle block removed: 240 steps in one launch, time per step
    (one wave on one CU: a latency figure, the GPU is nearly idle)."""
    scene = W.cfg1(0)
    stream = torch.cuda.current_stream()
    world = J.World(scene, stream=stream.cuda_stream)
    world.step(0)
    world.sync()
    _synced(J, J.jg_query_phase_cycles, world.h)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    world.step(240)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    phases = _synced(J, J.jg_query_phase_cycles, world.h)
    tot = max(1, sum(phases.values()))
    world.close()
    log(f"  removal tower: {ms / 240 * 1e3:.1f} us per step")
    return {"workload": "one 18-level tower (53 blocks after one middle block is removed), 240 steps",
            "us_per_step": ms / 240 * 1e3,
            "phase_cycle_share": {k: round(v / tot, 4) for k, v in phases.items()}}


def literal_tilt_rate(J, torch, W, steps):
    """The throughput batch with tilts of U(0, 3 deg) alone: the towers keep standing (resting
    contacts throughout)."""
    scene = W.cfg3(0, n_steps=steps, literal_tilt=True)
    v, ms, st = _run_timed(J, torch, scene, steps, run=RUN[0])
    log(f"  standing towers: {v:.4g} tower-steps/s")
    return {"workload": f"throughput batch with tilts of U(0, 3 deg): {scene['n_towers']} standing towers, "
                        f"{steps} steps", "value": v, "kernel_ms": ms, "error_word": int(st.error_word)}


def variants_ab(J, torch, W, towers=4096, steps=240, episode_steps=2000):
    """The solver variants against the literal solver (R36-R39):
    - disc friction;
    - restitution targets;
    - reference-face manifolds;
    - the paper's solver setting (14 sweeps, 3 substeps), on the same towers.

    Each variant runs two workloads:
    - the first `towers` towers of the throughput batch's recipe falling for `steps` steps: the
      rate, and the quartiles of each tower's centre-of-mass travel and drop (the collapse
      distributions);
    - the removal batch's episodes with the previous-step start: collapsed towers and withdrawn
      blocks per friction level.
    """
    import numpy as np
    from paper_2606_28394_amd import episodes as E
    fall = W.tilted_towers(3, towers, seed=31, n_steps=steps)
    ptr = np.asarray(fall["tower_ptr"])
    x0 = np.asarray(fall["pos"], np.float64).reshape(-1, 3)
    removal = W.cfg2(0, n_steps=episode_steps)
    # (name, solver parameters, world options); reference-face manifolds make collapsing towers
    # press more pairs together than the default 3.5 slots per body hold
    variants = (("literal", {}, {}), ("disc_friction", {"friction_cone": 1}, {}),
                ("restitution_targets", {"restitution_bias": 1}, {}),
                ("reference_face", {"manifold_mode": 1}, {"manifolds_per_body": 6.0}),
                ("paper_solver_14x3", {"iters": 14, "n_sub": 3}, {}))
    rows = []
    for name, over, kw in variants:
        sc = dict(fall, params=dict(fall["params"], **over))
        v, ms, st = _run_timed(J, torch, sc, steps, keep=True, run=RUN[0], **kw)
        world, st = st
        x = _synced(J, world.state)[0]
        world.close()
        d = np.stack([x[ptr[t]:ptr[t + 1]].mean(0) - x0[ptr[t]:ptr[t + 1]].mean(0) for t in range(len(ptr) - 1)])
        travel, drop = np.linalg.norm(d[:, :2], axis=1), -d[:, 2]
        rs = dict(removal, params=dict(removal["params"], **over))
        stream = torch.cuda.current_stream()
        ew = J.World(rs, warm_start=1, stream=stream.cuda_stream, **kw)
        ew.begin_episodes()
        ew.step(episode_steps)
        summ = E.summary(E.world_records(ew, rs))
        ew.close()
        row = {"variant": name, "tower_steps_per_s": v, "error_word": int(st.error_word),
               "travel_quartiles_m": [float(q) for q in np.quantile(travel, [.25, .5, .75])],
               "drop_quartiles_m": [float(q) for q in np.quantile(drop, [.25, .5, .75])],
               "episodes_collapsed": [r["collapsed"] for r in summ], "episodes_withdrawn": [r["removed"] for r in summ]}
        log(f"  {name}: {v:.4g} tower-steps/s, median travel {row['travel_quartiles_m'][1]:.3f} m, median drop "
            f"{row['drop_quartiles_m'][1]:.3f} m, collapsed {row['episodes_collapsed']}, withdrawn {row['episodes_withdrawn']}")
        rows.append(row)
    return {"workload": f"{towers} towers of the throughput batch's recipe falling {steps} steps; the removal batch's "
                        f"450 episodes ({episode_steps} steps, previous-step start; per mu {list(W.MU_LEVELS)})",
            "rows": rows}


def episodes_table(J, torch, W, steps=2000, warm_starts=(1, 0), out_dir=None):
    """The 450-episode experiment (Sec. "Effect of the Friction Coefficient", Tab. results) on the
    removal batch: every tower's episode (collapse criterion of Eq. (collapse), rest rule, moves of
    Tab. ziglar) on the GPU over one launch of `steps` steps.  Per friction level: collapsed episodes,
    mean rounds, Ziglar's thresholds F = k mu m g for the paper's block (19.6 g) and the benchmark
    block, the share of torque moves; and the three validation claims (collapses per move type, the
    trend with mu).  Run with the previous-step warm start and with the zero start."""
    import numpy as np
    from paper_2606_28394_amd import episodes as E
    scene = W.cfg2(0, n_steps=steps)
    T = scene["n_towers"]
    tower = W.tower_of(scene)
    out = {"workload": f"removal batch: {T} towers (150 per mu), 12-24 levels, 1-8 push removals, {steps} steps"}
    for ws in warm_starts:
        stream = torch.cuda.current_stream()
        world = J.World(scene, warm_start=ws, stream=stream.cuda_stream)
        world.begin_episodes()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        world.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        eps = [_synced(J, world.episode, t) for t in range(T)]
        records = E.world_records(world, scene)
        world.close()
        rows = E.summary(records)   # Tab. results, one row per friction level
        if out_dir:
            E.write_json(records, out_dir, tag=f"_{'previous_step' if ws == 1 else 'zero'}_start")
        by_move = {n: [0, 0] for n in W.MOVE_NAMES}      # collapses during a move of this type, moves
        moves_of = {}                                      # tower -> [(start, move)] of its moves
        for i in range(len(scene["push_body"])):
            mv = int(scene["push_move"][i])
            if mv >= 0:
                moves_of.setdefault(int(tower[int(scene["push_body"][i])]), []).append((int(scene["push_start"][i]), mv))
        for t, mvs in moves_of.items():
            e = eps[t]
            last = e.collapse_step if e.collapsed else steps - 1
            started = sorted(m for m in mvs if m[0] <= last)
            for _, mv in started:
                by_move[W.MOVE_NAMES[mv]][1] += 1
            # the move during which the collapse came: the last one started by the collapse step
            if e.collapsed and started:
                by_move[W.MOVE_NAMES[started[-1][1]]][0] += 1
        rates = {k: (v[0] / v[1] if v[1] else None) for k, v in by_move.items()}
        col_rate = [r["collapsed"] / r["episodes"] for r in rows]
        claims = {"side_yaxis_below_side_xaxis": None if None in (rates["side_yaxis"], rates["side_xaxis"])
                  else rates["side_yaxis"] < rates["side_xaxis"],
                  "center_safest": None if None in rates.values() else
                  rates["center_xaxis"] <= min(rates["side_yaxis"], rates["side_xaxis"]),
                  "collapse_rate_falls_with_mu": col_rate[0] >= col_rate[1] >= col_rate[2] and col_rate[0] > col_rate[2]}
        key = "previous_step_start" if ws == 1 else "zero_start"
        out[key] = {"kernel_ms": ms, "tower_steps_per_s": T * steps / (ms * 1e-3), "rows": rows,
                    "collapse_rate_by_move": rates, "moves_by_type": {k: v[1] for k, v in by_move.items()},
                    "ziglar_claims": claims}
        log(f"  episodes ({key}): collapsed {[r['collapsed'] for r in rows]} of 150, mean rounds "
            f"{[round(r['mean_rounds'], 2) for r in rows]}, {ms / steps:.3f} ms per step")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--towers", type=int, default=16384)
    ap.add_argument("--warm-start", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-towers", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=50)
    ap.add_argument("--learned-weights", default=DEFAULT_WEIGHTS,
                    help="trained warm-start network (.npy); the equal-residual leg runs when it exists")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--cpu-report", action="store_true",
                    help="also time the oracle single-threaded and on all host threads over samples of "
                         "every workload (a few minutes)")
    ap.add_argument("--episodes-json", default=None, metavar="DIR",
                    help="write the episode records and per-friction summaries of the episode leg as JSON")
    ap.add_argument("--no-episodes", action="store_true",
                    help="skip the 450-episode table (collapse criterion and labels on the removal batch)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-tower latency and standing-tower legs")
    ap.add_argument("--island-steps", type=int, default=100,
                    help="steps of the large-island leg (one 64 x 64 masonry wall); 0 skips it and the "
                         "wall's equal-residual leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's pack size instead of timing candidates on the batch first")
    ap.add_argument("--tune-steps", type=int, default=40,
                    help="steps timed per candidate pack size (after a 60-step lead-in)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first copy MB megabytes device to device once (a known-size reference for "
                         "profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); towers shard across GPUs with no "
              "exchange, so a multi-GPU run would be N independent copies of this one", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_28394_amd import jenga as J
    from paper_2606_28394_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    J.load_library()
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 4} bytes read and written once")
        del src, dst
    log("generating the batch ...")
    t0 = time.perf_counter()
    scene = W.cfg3(0, n_towers=args.towers, n_steps=args.steps)
    log(f"  {scene['n_towers']} towers, {int(scene['tower_ptr'][-1])} bodies in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    pack_bodies, tuned = 0, None
    if not args.no_autotune:
        from paper_2606_28394_amd import autotune as A
        log("pack-size tuner ...")
        t0 = time.perf_counter()
        tuned = A.tune_pack_bodies(scene, steps=args.tune_steps, lead_in=60, warm_start=args.warm_start, log=log)
        pack_bodies = tuned["pack_bodies"]
        log(f"  chose pack_bodies {pack_bodies} in {time.perf_counter() - t0:.1f} s")
    world = J.World(scene, warm_start=args.warm_start, stream=stream.cuda_stream, pack_bodies=pack_bodies)
    sizes = np.diff(scene["tower_ptr"]).tolist()
    init = world.state()

    if args.warmup > 0:
        world.step(args.warmup)
        _synced(J, world.sync)
        log(f"warm-up {args.warmup} steps done")
        world.set_state(*init)
    world.step(0)          # make the restored state resident before the timed region
    _synced(J, world.sync)
    s0 = _synced(J, world.stats)
    _synced(J, J.jg_query_phase_cycles, world.h)   # reset the per-phase counters

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    world.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1)
    s1 = _synced(J, world.stats)
    phases = _synced(J, J.jg_query_phase_cycles, world.h)
    total_cyc = max(1, sum(phases.values()))
    log(f"timed {args.steps} steps: wall {wall * 1e3:.1f} ms, kernel (events) {kernel_ms:.1f} ms")
    log("phase share of workgroup cycles: " + ", ".join(f"{k} {100.0 * v / total_cyc:.1f}%" for k, v in phases.items()))

    T = scene["n_towers"]
    cand = s1.candidates - s0.candidates
    man = s1.manifolds - s0.manifolds
    pts = s1.points - s0.points
    ci = s1.contact_iters - s0.contact_iters
    tower_steps = T * args.steps
    value = tower_steps / wall
    flops = algorithmic_flops(sizes, args.steps, cand, man, pts, 20)
    achieved_tflops = flops / (kernel_ms * 1e-3) / 1e12
    workload = f"throughput batch: {T} tilted towers, 8-40 levels x 3 boxes, {args.steps} steps"
    traffic = traffic_from_profile(kernel_hash(), workload, args.steps, pack_bodies)
    last_points = pts / max(1, args.steps)
    bytes_launch = algorithmic_bytes(int(scene["tower_ptr"][-1]), last_points)
    out = {
        "metric": "tower-steps/s",
        "value": value,
        "unit": "tower-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "towers": T, "bodies": int(scene["tower_ptr"][-1]),
                   "pgs_iters": 20, "dt": 1 / 240, "warm_start": "previous step" if args.warm_start else "zero",
                   "launch": "one persistent launch of all steps, one 64-lane workgroup per pack of towers, "
                             "packs grouped by workgroups per CU into launch classes that run side by side",
                   "pack_bodies": pack_bodies if pack_bodies else "library default",
                   "pack_tuning": None if tuned is None else
                   {"tower_steps_per_s": tuned["tower_steps_per_s"], "steps": tuned["steps"],
                    "lead_in": tuned["lead_in"], "margin": tuned["margin"]}},
        "contact_iters_per_s": ci / wall,
        "kernel_ms": kernel_ms,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "hbm_algorithmic_gbs": bytes_launch / (kernel_ms * 1e-3) / 1e9,
                     "hbm_measured_gbs": None if traffic is None else traffic / (kernel_ms * 1e-3) / 1e9,
                     # both components of max(B / 8 TB/s, F / 157.3 TF) / time
                     "alu_frac": achieved_tflops / PEAK_FP32_TFLOPS,
                     "hbm_frac_algorithmic": bytes_launch / (kernel_ms * 1e-3) / (PEAK_HBM_GBS * 1e9),
                     "hbm_frac_measured": None if traffic is None else traffic / (kernel_ms * 1e-3) / (PEAK_HBM_GBS * 1e9)},
        "phase_cycle_share": {k: round(v / total_cyc, 4) for k, v in phases.items()},
        "error_word": int(s1.error_word),
        "residual_rms_max": s1.residual_rms,
    }
    # the same batch while it collapses (dense dynamic contacts): untimed steps up to step 200 after
    # the timed window, then the same number of timed steps again
    lead = max(0, 200 - args.steps)
    if lead:
        world.step(lead)
        _synced(J, world.sync)
    n2 = max(20, args.steps)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record(stream)
    world.step(n2)
    ev3.record(stream)
    torch.cuda.synchronize()
    ms2 = ev2.elapsed_time(ev3)
    first = args.steps + lead + 1
    out["collapse_phase"] = {"steps": f"{first}-{first + n2 - 1}", "tower_steps_per_s": T * n2 / (ms2 * 1e-3),
                             "kernel_ms": ms2, "error_word": int(_synced(J, world.stats).error_word)}
    log(f"collapse phase (steps {first}-{first + n2 - 1}): {T * n2 / (ms2 * 1e-3):.4g} tower-steps/s")
    world.close()
    if not args.no_extra:
        log("single-tower latency and standing-tower legs ...")
        RUN[0] = "single tower"
        out["single_tower"] = single_tower_latency(J, torch, W)
        RUN[0] = "standing towers"
        out["standing_towers"] = literal_tilt_rate(J, torch, W, args.steps)
        log("solver variants A/B ...")
        RUN[0] = "variants A/B"
        out["variants_ab"] = variants_ab(J, torch, W)
    if not args.no_episodes:
        log("episode table (removal batch) ...")
        RUN[0] = "episodes"
        out["episodes"] = episodes_table(J, torch, W, out_dir=args.episodes_json)
    if args.island_steps > 0:
        log("large-island leg (64 x 64 masonry wall) ...")
        RUN[0] = "large island"
        out["large_island"] = large_island(J, torch, W, args.island_steps)
        log("grid-wide islands (100,000-stone wall; the 4,096-stone wall on the same path) ...")
        RUN[0] = "grid-wide islands"
        out["grid_wide_islands"] = grid_wide_islands(J, torch, W)
    if not args.no_learned and os.path.exists(args.learned_weights):
        log("equal-residual leg (learned warm start vs plain-20) ...")
        out["equal_residual"] = equal_residual(J, torch, args.learned_weights)
        if args.island_steps > 0:
            log("equal-residual leg on the 64 x 64 masonry wall ...")
            out["equal_residual_wall"] = equal_residual(
                J, torch, args.learned_weights, steps=300, ks=(1, 2, 3, 4), scene=W.cfg5(0, n_steps=300),
                workload="one masonry wall, 64 courses x 64 stones (4096 bodies), steps 1-300")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_towers, args.cpu_steps)
    if args.cpu_report:
        log("oracle timing report ...")
        out["cpu_report"] = cpu_report()
    out["device_error_reports"] = DEVICE_ERRORS
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
