"""Seeded synthetic workloads: towers of oriented boxes, as plain input arrays.

This module only builds inputs (geometry, masses, initial state, friction per
tower, push schedules).  It holds none of the stepping arithmetic, so both the
FP64 oracle and the HIP path read exactly the same scene.

Tower construction follows the paper's structural constraints (Sec. "Structural
Constraints": three blocks per layer, alternating perpendicular layers, block
ratios L = 3W, T = 0.6W) with the block size and density of the benchmark
configurations (75 x 25 x 15 mm, 600 kg/m^3).  Push magnitudes are multiples of
Ziglar's thresholds F = k mu m g (Eq. 4, k = 3; Eq. 8, k = 4).

Every random draw comes from ``numpy.random.default_rng([260628394, config_id,
tower_index])`` so that any tower of any configuration can be regenerated alone.

A scene is a dict of numpy arrays:
  n_towers            int
  tower_ptr  (T+1,)   int64   bodies of tower t are [tower_ptr[t], tower_ptr[t+1])
  half_extents (N,3)  f64     body-frame half sizes (x = length, y = width, z = thickness)
  mass       (N,)     f64     0 => static body
  pos (N,3), quat (N,4) [w,x,y,z], linvel (N,3), angvel (N,3) (world frame)
  active     (N,)     u8
  mu         (T,)     f64     static friction coefficient of each tower
  push_body  (K,)     int32   global body index
  push_force (K,3)    f64     constant world-frame force [N]
  push_start (K,)     int32   first step the force acts
  push_steps (K,)     int32   number of steps it acts
  push_withdraw (K,)  f64     displacement along the force that deactivates the body (0 = never)
  push_move  (K,)     int32   the move a push is (Tab. ziglar): MOVE_CENTER_X, MOVE_SIDE_Y, MOVE_SIDE_X,
                              or -1 when the push is not a block removal
  params     dict     dt, iters, n_sub, restitution, beta, slop, margin, gravity, friction_cone (0 per-axis
                      clip, 1 disc), restitution_bias (0 as printed, 1 pre-solve target), manifold_mode
                      (0 literal silhouettes, 1 reference-face clipping)
  n_steps    int      steps the configuration runs
"""
from __future__ import annotations

import math

import numpy as np

SEED_ROOT = 260628394

# Benchmark block: 75 x 25 x 15 mm, density 600 kg/m^3 -> 16.875 g.
BLOCK_HALF = np.array([0.0375, 0.0125, 0.0075])
BLOCK_DENSITY = 600.0
BLOCK_MASS = BLOCK_DENSITY * float(np.prod(2.0 * BLOCK_HALF))
# The paper's block (appendix table): 81 x 26 x 18 mm, 19.6 g.
PAPER_BLOCK_HALF = np.array([0.0405, 0.013, 0.009])
PAPER_BLOCK_MASS = 0.0196

G = 9.81
MU_LEVELS = (0.25, 0.40, 0.60)
# the move types of Tab. ziglar (which block, which axis), with Ziglar's force factor k
MOVE_CENTER_X, MOVE_SIDE_Y, MOVE_SIDE_X = 0, 1, 2
MOVE_NAMES = ("center_xaxis", "side_yaxis", "side_xaxis")
MOVE_K = (3, 3, 4)
LAYER_GAP = 1e-3        # in-layer gap between neighbouring blocks
BED_OVERLAP = 1e-4      # initial vertical overlap (keeps resting contacts active)
JITTER = 5e-4           # horizontal placement jitter (uniform +-)


def default_params(**over):
    p = dict(dt=1.0 / 240.0, iters=20, n_sub=1, restitution=0.10, beta=0.35,
             slop=4e-4, margin=2e-3, gravity=(0.0, 0.0, -G), friction_cone=0, restitution_bias=0,
             manifold_mode=0, mega_bodies=16384, colour_partition=1024)
    p.update(over)
    return p


def rng_for(config_id: int, index: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(config_id), int(index)])


def quat_z(angle: float) -> np.ndarray:
    return np.array([math.cos(angle / 2), 0.0, 0.0, math.sin(angle / 2)])


def quat_axis_angle(axis, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    s = math.sin(angle / 2)
    return np.array([math.cos(angle / 2), a[0] * s, a[1] * s, a[2] * s])


def quat_mul(a, b) -> np.ndarray:
    """Hamilton product (placement helper only: used to build initial poses)."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _rotate(q, v) -> np.ndarray:
    """Rotate vector v by unit quaternion q (placement helper only)."""
    w, x, y, z = q
    u = np.array([x, y, z])
    v = np.asarray(v, dtype=np.float64)
    return v + 2.0 * np.cross(u, np.cross(u, v) + w * v)


def jenga_tower(levels: int, rng: np.random.Generator | None, half=BLOCK_HALF,
                mass=None, jitter=JITTER):
    """One upright tower: ``levels`` layers of 3 blocks, alternating 90 deg.

    Level l has its long axis along world x when l is even, y when odd; the
    three slots sit at -(w+gap), 0, +(w+gap) across the long axis.  Layers
    overlap by 0.1 mm so resting contacts are active from step 0.
    Returns (half_extents, mass, pos, quat, level, slot).
    """
    half = np.asarray(half, dtype=np.float64)
    if mass is None:
        mass = BLOCK_DENSITY * float(np.prod(2.0 * half))
    width = 2.0 * half[1]
    thick = 2.0 * half[2]
    n = 3 * levels
    he = np.tile(half, (n, 1))
    m = np.full(n, float(mass))
    lev = np.repeat(np.arange(levels, dtype=np.int32), 3)
    slot = np.tile(np.arange(3, dtype=np.int32), levels)
    if rng is not None and jitter > 0:
        jit = rng.uniform(-jitter, jitter, size=(n, 2))    # drawn per block in tower order
    else:
        jit = np.zeros((n, 2))
    along_x = (lev % 2 == 0)
    off = (slot - 1) * (width + LAYER_GAP)
    z = half[2] - BED_OVERLAP + lev * (thick - BED_OVERLAP)
    pos = np.stack([np.where(along_x, jit[:, 0], off + jit[:, 0]),
                    np.where(along_x, off + jit[:, 1], jit[:, 1]), z], 1)
    q90 = quat_z(math.pi / 2)
    quat = np.where(along_x[:, None], np.array([1.0, 0.0, 0.0, 0.0]), q90)
    return he, m, pos, quat, lev, slot


_EDGE_DIRS = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
_SIGNS = np.array([[1 if c & 1 else -1, 1 if c & 2 else -1, 1 if c & 4 else -1] for c in range(8)], float)


def _rot_matrices(quat) -> np.ndarray:
    """Rotation matrices of unit quaternions (placement helper only)."""
    w, x, y, z = (np.asarray(quat, np.float64)[:, k] for k in range(4))
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], -2)


def _all_corners(pos, quat, he) -> np.ndarray:
    R = _rot_matrices(quat)
    local = _SIGNS[None, :, :] * np.asarray(he)[:, None, :]
    return np.asarray(pos)[:, None, :] + np.einsum("nij,nkj->nki", R, local)


def _pivot(pos, quat, he, edge):
    d = _EDGE_DIRS[edge]
    c = _all_corners(pos, quat, he).reshape(-1, 3)
    return d, float((c @ d).max()), float(c[:, 2].min())


def tilt_about_edge(pos, quat, he, theta: float, edge: int):
    """Rigidly rotate a tower by ``theta`` about one bottom edge of its footprint.

    edge in {0: +x, 1: -x, 2: +y, 3: -y} picks the footprint side the tower
    tips towards.  Returns new (pos, quat).
    """
    d, ext, zmin = _pivot(pos, quat, he, edge)
    pivot = d * ext + np.array([0.0, 0.0, zmin])
    axis = np.cross(np.array([0.0, 0.0, 1.0]), d)
    qr = quat_axis_angle(axis, theta)
    Rr = _rot_matrices(qr[None, :])[0]
    npos = pivot + (np.asarray(pos) - pivot) @ Rr.T
    aw, ax, ay, az = qr
    bw, bx, by, bz = (np.asarray(quat)[:, k] for k in range(4))
    nquat = np.stack([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                      aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw], 1)
    return npos, nquat


def critical_tilt(pos, quat, he, edge: int) -> float:
    """Tilt at which the tower's centre of mass sits above the pivot edge."""
    d, ext, zmin = _pivot(pos, quat, he, edge)
    com = np.asarray(pos).mean(axis=0)
    return math.atan2(ext - float(d @ com), float(com[2]) - zmin)


class SceneBuilder:
    """Accumulates towers and pushes into one scene dict."""

    def __init__(self, params=None, n_steps=1):
        self.params = params or default_params()
        self.n_steps = n_steps
        self.towers = []     # list of dicts of body arrays
        self.mu = []
        self.pushes = []     # (global body, force, start, steps, withdraw)
        self.n_bodies = 0

    def add_tower(self, he, m, pos, quat, mu, linvel=None, angvel=None, active=None, level=None, slot=None):
        """level, slot: each block's layer and position in it (a tower built by jenga_tower), kept
        for the episode labels' map of removed positions; -1 where not given."""
        n = len(m)
        t = dict(he=np.asarray(he, np.float64).reshape(n, 3),
                 m=np.asarray(m, np.float64).reshape(n),
                 pos=np.asarray(pos, np.float64).reshape(n, 3),
                 quat=np.asarray(quat, np.float64).reshape(n, 4),
                 v=np.zeros((n, 3)) if linvel is None else np.asarray(linvel, np.float64).reshape(n, 3),
                 w=np.zeros((n, 3)) if angvel is None else np.asarray(angvel, np.float64).reshape(n, 3),
                 active=np.ones(n, np.uint8) if active is None else np.asarray(active, np.uint8).reshape(n),
                 level=np.full(n, -1, np.int32) if level is None else np.asarray(level, np.int32).reshape(n),
                 slot=np.full(n, -1, np.int32) if slot is None else np.asarray(slot, np.int32).reshape(n))
        first = self.n_bodies
        self.towers.append(t)
        self.mu.append(float(mu))
        self.n_bodies += n
        return first

    def add_push(self, body, force, start, steps, withdraw=0.0, move=-1):
        self.pushes.append((int(body), np.asarray(force, np.float64).reshape(3), int(start), int(steps),
                            float(withdraw), int(move)))

    def build(self):
        T = len(self.towers)
        ptr = np.zeros(T + 1, np.int64)
        for i, t in enumerate(self.towers):
            ptr[i + 1] = ptr[i] + len(t["m"])
        cat = lambda k: np.concatenate([t[k] for t in self.towers]) if T else np.zeros(0)
        K = len(self.pushes)
        sc = dict(
            n_towers=T, tower_ptr=ptr,
            half_extents=cat("he").reshape(-1, 3), mass=cat("m"), pos=cat("pos").reshape(-1, 3),
            quat=cat("quat").reshape(-1, 4), linvel=cat("v").reshape(-1, 3), angvel=cat("w").reshape(-1, 3),
            active=cat("active").astype(np.uint8), mu=np.asarray(self.mu, np.float64),
            body_level=cat("level").astype(np.int32), body_slot=cat("slot").astype(np.int32),
            push_body=np.array([p[0] for p in self.pushes], np.int32).reshape(K),
            push_force=np.array([p[1] for p in self.pushes], np.float64).reshape(K, 3),
            push_start=np.array([p[2] for p in self.pushes], np.int32).reshape(K),
            push_steps=np.array([p[3] for p in self.pushes], np.int32).reshape(K),
            push_withdraw=np.array([p[4] for p in self.pushes], np.float64).reshape(K),
            push_move=np.array([p[5] for p in self.pushes], np.int32).reshape(K),
            params=dict(self.params), n_steps=int(self.n_steps))
        return sc


def tower_of(scene) -> np.ndarray:
    ptr = scene["tower_ptr"]
    return np.repeat(np.arange(scene["n_towers"], dtype=np.int32), np.diff(ptr))


def subset(scene, towers) -> dict:
    """Scene restricted to the listed towers (pushes re-indexed)."""
    towers = list(towers)
    ptr = scene["tower_ptr"]
    sb = SceneBuilder(scene["params"], scene["n_steps"])
    remap = {}
    for t in towers:
        a, b = int(ptr[t]), int(ptr[t + 1])
        first = sb.add_tower(scene["half_extents"][a:b], scene["mass"][a:b], scene["pos"][a:b],
                             scene["quat"][a:b], scene["mu"][t], scene["linvel"][a:b],
                             scene["angvel"][a:b], scene["active"][a:b],
                             scene["body_level"][a:b] if "body_level" in scene else None,
                             scene["body_slot"][a:b] if "body_slot" in scene else None)
        for k in range(a, b):
            remap[k] = first + (k - a)
    for i in range(len(scene["push_body"])):
        b = int(scene["push_body"][i])
        if b in remap:
            sb.add_push(remap[b], scene["push_force"][i], scene["push_start"][i], scene["push_steps"][i],
                        scene["push_withdraw"][i], int(scene["push_move"][i]) if "push_move" in scene else -1)
    return sb.build()


# ----------------------------------------------------------------------------------------------
# Benchmark configurations
# ----------------------------------------------------------------------------------------------

def paper_preset_params(**over):
    """The paper's own simulator settings (appendix "Physical Parameters"): 14 PGS iterations and
    three substeps of a 1/240 s step."""
    return default_params(iters=14, n_sub=3, **over)


def paper_tower(levels: int, rng: np.random.Generator | None):
    """A tower of the paper's block (81 x 26 x 18 mm, 19.6 g), same layout recipe."""
    return jenga_tower(levels, rng, half=PAPER_BLOCK_HALF, mass=PAPER_BLOCK_MASS)


def cfg1(seed: int = 0):
    """One 18-level tower (54 blocks), one seeded middle block removed at t = 0.

    mu = 0.40, 20 iterations, dt = 1/240 s, 240 steps.
    """
    rng = rng_for(1, seed)
    he, m, pos, quat, lev, slot = jenga_tower(18, rng)
    active = np.ones(len(m), np.uint8)
    level = int(rng.integers(8, 10))
    s = int(rng.integers(0, 3))
    active[3 * level + s] = 0
    sb = SceneBuilder(default_params(), n_steps=240)
    sb.add_tower(he, m, pos, quat, 0.40, active=active, level=lev, slot=slot)
    return sb.build()


def _tower_push_schedule(rng, levels, mu, first_body, sb, n_removals):
    """Seeded removals: at step 60 + 240 r push one block (levels 1..L-3) for 180 steps."""
    chosen = set()
    for r in range(n_removals):
        while True:
            l = int(rng.integers(1, levels - 2))
            s = int(rng.integers(0, 3))
            if (l, s) not in chosen:
                chosen.add((l, s))
                break
        along_x = (l % 2 == 0)
        long_axis = np.array([1.0, 0, 0]) if along_x else np.array([0, 1.0, 0])
        short_axis = np.array([0, 1.0, 0]) if along_x else np.array([1.0, 0, 0])
        # the centre block leaves along its length ("center_xaxis"); a side block along its length
        # ("side_yaxis") or outwards across it ("side_xaxis", the torque move)
        if s == 1 or rng.random() < 0.5:
            move, direction, extent = (MOVE_CENTER_X if s == 1 else MOVE_SIDE_Y), \
                long_axis * (1 if rng.random() < 0.5 else -1), 2 * BLOCK_HALF[0]
        else:
            move, direction, extent = MOVE_SIDE_X, short_axis * (1 if s == 2 else -1), 2 * BLOCK_HALF[1]
        scale = rng.uniform(0.9, 1.3)
        f = scale * MOVE_K[move] * mu * BLOCK_MASS * G
        sb.add_push(first_body + 3 * l + s, f * direction, 60 + 240 * r, 180, extent, move)


def cfg2(seed: int = 0, n_per_mu: int = 150, n_steps: int = 2000):
    """450 towers (150 per mu level), 12-24 levels, 1-8 seeded push removals each."""
    sb = SceneBuilder(default_params(), n_steps=n_steps)
    idx = 0
    for mu in MU_LEVELS:
        for _ in range(n_per_mu):
            rng = rng_for(2, seed * 100000 + idx)
            levels = int(rng.integers(12, 25))
            he, m, pos, quat, lev, slot = jenga_tower(levels, rng)
            first = sb.add_tower(he, m, pos, quat, mu, level=lev, slot=slot)
            _tower_push_schedule(rng, levels, mu, first, sb, int(rng.integers(1, 9)))
            idx += 1
    return sb.build()


def cfg3(seed: int = 0, n_towers: int = 16384, n_steps: int = 500, literal_tilt: bool = False,
         min_levels: int = 8, max_levels: int = 40):
    """Throughput batch: towers of 8-40 levels, each tilted past its critical angle.

    The tilt is theta_crit(L) + U(0, 3 deg) about a seeded bottom edge, so every
    tower collapses fully (dense, dynamic contacts).  ``literal_tilt`` draws the
    tilt from U(0, 3 deg) alone (towers keep standing).
    """
    sb = SceneBuilder(default_params(), n_steps=n_steps)
    for t in range(n_towers):
        rng = rng_for(3, seed * 1000000 + t)
        levels = int(rng.integers(min_levels, max_levels + 1))
        mu = MU_LEVELS[int(rng.integers(0, 3))]
        he, m, pos, quat, lev, slot = jenga_tower(levels, rng)
        edge = int(rng.integers(0, 4))
        extra = math.radians(rng.uniform(0.0, 3.0))
        theta = extra if literal_tilt else critical_tilt(pos, quat, he, edge) + extra
        pos, quat = tilt_about_edge(pos, quat, he, theta, edge)
        sb.add_tower(he, m, pos, quat, mu)
    return sb.build()


def tilted_towers(config_id: int, n_towers: int, levels_range=(8, 40), seed: int = 0, n_steps: int = 1,
                  literal_tilt: bool = False):
    """Smaller batches with the same recipe as the throughput batch (for parity tests)."""
    sb = SceneBuilder(default_params(), n_steps=n_steps)
    for t in range(n_towers):
        rng = rng_for(config_id, seed * 1000000 + t)
        levels = int(rng.integers(levels_range[0], levels_range[1] + 1))
        mu = MU_LEVELS[int(rng.integers(0, 3))]
        he, m, pos, quat, lev, slot = jenga_tower(levels, rng)
        edge = int(rng.integers(0, 4))
        extra = math.radians(rng.uniform(0.0, 3.0))
        theta = extra if literal_tilt else critical_tilt(pos, quat, he, edge) + extra
        pos, quat = tilt_about_edge(pos, quat, he, theta, edge)
        sb.add_tower(he, m, pos, quat, mu)
    return sb.build()


def random_box_pairs(n: int, seed: int = 0, size=(0.1, 1.0), spread=1.5):
    """Random box pairs (for separating-axis checks): half extents, centres, unit quaternions."""
    rng = rng_for(90, seed)
    he = rng.uniform(size[0], size[1], size=(n, 2, 3)) / 2.0
    x = rng.uniform(-spread / 2, spread / 2, size=(n, 2, 3))
    q = rng.normal(size=(n, 2, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    return he, x, q


def single_box(pos, quat=(1.0, 0, 0, 0), linvel=(0, 0, 0), angvel=(0, 0, 0), half=BLOCK_HALF,
               mass=BLOCK_MASS, mu=0.4, params=None, n_steps=1):
    sb = SceneBuilder(params or default_params(), n_steps=n_steps)
    sb.add_tower([half], [mass], [pos], [quat], mu, [linvel], [angvel])
    return sb.build()


def mlp_init(seed: int = 0, n_feat: int = 24, hidden: int = 128, n_out: int = 3) -> np.ndarray:
    """Initial parameters of the per-contact warm-start network, flat float64 in the order
    W1[n_feat][hidden], b1, W2[hidden][hidden], b2, W3[hidden][n_out], b3, mean[n_feat], std[n_feat].
    Weights and biases are uniform in +-1/sqrt(fan_in); mean 0 and std 1 (identity normalisation)."""
    rng = rng_for(41, seed)
    parts = []
    for fan_in, fan_out in ((n_feat, hidden), (hidden, hidden), (hidden, n_out)):
        bound = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, fan_in * fan_out))
        parts.append(rng.uniform(-bound, bound, fan_out))
    parts.append(np.zeros(n_feat))
    parts.append(np.ones(n_feat))
    return np.concatenate(parts)


def random_features(n: int, seed: int = 0, n_feat: int = 24) -> np.ndarray:
    """Feature-shaped random rows (standard normal), for network tests."""
    return rng_for(42, seed).standard_normal((n, n_feat))


STONE_DENSITY = 2400.0


def masonry_wall(courses: int = 64, per_course: int = 64, seed: int = 0, n_steps: int = 3000,
                 shear: float = 0.5, mu: float = 0.60, params=None) -> dict:
    """One wall of stones in running bond, as one island (one tower of the scene).

    Stone length ~ LogNormal(ln 0.3, 0.25) [m]; each course draws an aspect a_c ~ U(1, 3) and
    has height 0.3 / a_c; depth (through the wall) 0.3 m; 1 mm head joints; odd courses start
    0.15 m further along x (running bond); courses overlap by 0.1 mm so the bed contacts are
    active from the first step; density 2400 kg/m^3.  The bottom course starts with velocity
    `shear` m/s along x (an in-plane base shear)."""
    rng = rng_for(5, seed)
    depth = 0.3
    he, m, pos, vel = [], [], [], []
    z = 0.0
    for c in range(courses):
        a_c = rng.uniform(1.0, 3.0)
        h = 0.3 / a_c
        lengths = np.exp(rng.normal(math.log(0.3), 0.25, per_course))
        x = 0.15 if c % 2 else 0.0
        zc = z + h / 2 - BED_OVERLAP
        for k in range(per_course):
            L = float(lengths[k])
            half = np.array([L / 2, depth / 2, h / 2])
            he.append(half)
            m.append(STONE_DENSITY * L * depth * h)
            pos.append([x + L / 2, 0.0, zc])
            vel.append([shear if c == 0 else 0.0, 0.0, 0.0])
            x += L + LAYER_GAP
        z = zc + h / 2
    n = len(m)
    sb = SceneBuilder(params or default_params(), n_steps=n_steps)
    sb.add_tower(np.array(he), np.array(m), np.array(pos), np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), mu,
                 np.array(vel), np.zeros((n, 3)))
    return sb.build()


def cfg5(seed: int = 0, n_steps: int = 3000):
    """The masonry collapse: one wall of 64 courses x 64 stones (4096 bodies, one island)."""
    return masonry_wall(64, 64, seed=seed, n_steps=n_steps)
